// Batched stepping of independent 2D periodic grids (each with its own size,
// time step and coefficients; no current; a fixed number m of sweeps).
//
// Every grid is cut into work items exactly as a single-grid launch would
// cut it (strips of columns x chunks of rows), and the items of all grids
// are concatenated: item it belongs to grid g with items[g] <= it <
// items[g+1].  Two schedules:
//  * grouped: one launch per phase (front, then each sweep pass) covering
//    the items of every grid;
//  * persistent: one cooperative launch runs all steps; workgroups claim
//    items from an atomic counter (so uneven items balance), and an item
//    waits only for the previous phase of its own grid (per-grid counters,
//    no grid-wide barrier).  The wait is bounded: on time-out it raises an
//    error flag and every workgroup leaves, so the launch always drains.
// In FP32 the front and the first sweep pass run as one phase (the fused
// pass of k2fs_impl.h, on the front's work items, whose 224-column aligned
// strips are the fused pass's own), so a step has one phase fewer.
#pragma once

#include "k2f_impl.h"
#include "k2fs_impl.h"
#include "k2s_impl.h"

namespace mx {
namespace batch2d {

constexpr int RX = STRIP;

// largest g with items[g] <= it, items[0] = 0, items[ng] = total.  The
// result is the same in every lane (it is); read from the first lane it is
// a scalar, so the grid descriptor's loads are scalar too.
__device__ __forceinline__ int find_grid(const int *items, int ng, int it)
{
    int lo = 0, hi = ng;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (items[mid] <= it) lo = mid; else hi = mid;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

template <typename T>
__device__ __forceinline__ void front_item(const GridDesc<T> *d, int ng, const int *items, int L, int bin, int it,
                                           void *lds, double *sred)
{
    const int g = find_grid(items, ng, it);
    const GridDesc<T> &gd = d[g];
    // the coefficients as values: through a reference into global memory
    // the compiler would reload them after every store of a field
    const Coef<T> c = gd.c;
    FrontArgs<T> fa;
    for (int q = 0; q < 3; q++) {
        fa.E[q] = gd.E[q];
        fa.B[q] = gd.B[bin ^ 1][q];
        fa.J0[q] = nullptr;
        fa.dEp[q] = gd.dEp[q];
    }
    fa.env_src = T(0);
    fa.partial = nullptr;
    front2d::front_tile<T, 3, 0, RX, false>(c, fa, gd.B[bin][0], gd.B[bin][1], gd.B[bin][2], L, gd.nsx_f,
                                            it - items[g], 0, lds, sred);
}

// the front and the first pass of K sweeps (writes iterate buffer 0)
template <typename T, int K>
__device__ __forceinline__ void front_sweep_item(const GridDesc<T> *d, int ng, const int *items, int L, int bin,
                                                 int it, void *lds)
{
    const int g = find_grid(items, ng, it);
    const GridDesc<T> &gd = d[g];
    // the coefficients as values: through a reference into global memory
    // the compiler would reload them after every store of a field
    const Coef<T> c = gd.c;
    FrontArgs<T> fa;
    SweepArgs<T> sa;
    for (int q = 0; q < 3; q++) {
        fa.E[q] = gd.E[q];
        fa.B[q] = gd.B[bin ^ 1][q];
        fa.J0[q] = nullptr;
        fa.dEp[q] = gd.dEp[q];
        sa.rhs[q] = gd.dEp[q];
        sa.x_in[q] = gd.dEp[q];
        sa.s_in[q] = nullptr;
        sa.x_out[q] = gd.X[0][q];
        sa.s_out[q] = nullptr;
        sa.E[q] = nullptr;
    }
    fa.env_src = T(0);
    fa.partial = nullptr;
    sa.partial = nullptr;
    sa.skip = nullptr;
    static_assert(fused2d::fs_width<0, K, RX, true>() == STRIP - 32, "fused strips are the front's strips");
    fused2d::fs_tile<T, 0, K, RX, false, true, 1>(c, fa, gd.B[bin][0], gd.B[bin][1], gd.B[bin][2], sa, L,
                                                  gd.nsx_f, it - items[g], lds);
}

template <typename T, int K, int OM>
__device__ __forceinline__ void sweep_item(const GridDesc<T> *d, int ng, const int *items, int L, bool first,
                                           int xin, int xout, int it, void *lds, double *sred)
{
    const int g = find_grid(items, ng, it);
    const GridDesc<T> &gd = d[g];
    // the coefficients as values: through a reference into global memory
    // the compiler would reload them after every store of a field
    const Coef<T> c = gd.c;
    SweepArgs<T> sa;
    for (int q = 0; q < 3; q++) {
        sa.rhs[q] = gd.dEp[q];
        sa.x_in[q] = first ? gd.dEp[q] : gd.X[xin][q];
        sa.s_in[q] = nullptr;
        sa.x_out[q] = gd.X[xout][q];
        sa.s_out[q] = nullptr;
        sa.E[q] = gd.E[q];
    }
    sa.partial = nullptr;
    sa.skip = nullptr;
    stream2d::stream_tile<T, 3, K, false, RX, OM>(c, sa, first ? SW_FIRST : 0, L, gd.nsx_s, it - items[g], 0,
                                                  lds, sred);
}

template <typename T>
__global__ __launch_bounds__(RX) void kb_front(const GridDesc<T> *d, int ng, const int *items, int L, int bin)
{
    __shared__ __attribute__((aligned(16))) char lds[front2d::front_lds_bytes<T, 0, RX>()];
    __shared__ double sred[2 * RX / 64];
    front_item<T>(d, ng, items, L, bin, xcd_map(blockIdx.x, gridDim.x), lds, sred);
}

template <typename T, int K>
__global__ __launch_bounds__(RX) void kb_front_sweep(const GridDesc<T> *d, int ng, const int *items, int L, int bin)
{
    __shared__ __attribute__((aligned(16))) char lds[fused2d::fs_lds_bytes<T, 0, K, RX>()];
    front_sweep_item<T, K>(d, ng, items, L, bin, xcd_map(blockIdx.x, gridDim.x), lds);
}

template <typename T, int K, int OM>
__global__ __launch_bounds__(RX) void kb_sweep(const GridDesc<T> *d, int ng, const int *items, int L, int first,
                                               int xin, int xout)
{
    __shared__ __attribute__((aligned(16))) char lds[stream2d::stream_lds_bytes<T, 3, K, RX>()];
    __shared__ double sred[2 * RX / 64];
    sweep_item<T, K, OM>(d, ng, items, L, first != 0, xin, xout, xcd_map(blockIdx.x, gridDim.x), lds, sred);
}

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }

// the fused first pass of a persistent kernel whose passes are Q - 1 or Q
// deep: FP32, and a depth with a fused kernel (no LDS when none)
template <typename T, int K>
constexpr bool fuse_k() { return sizeof(T) == 4 && K >= FUSE_KMIN && K <= FUSE_KMAX; }
template <typename T, int Q>
constexpr bool fuse_q() { return fuse_k<T, Q - 1>() || fuse_k<T, Q>(); }
template <typename T, int K>
constexpr size_t fuse_lds() { if constexpr (fuse_k<T, K>()) return fused2d::fs_lds_bytes<T, 0, K, RX>(); else return 0; }

// The persistent schedule: all nsteps steps of all grids in one cooperative
// launch; npass passes per step, the first nlow of Q - 1 sweeps, the others
// of Q (FUSE: the front and the first pass run as one phase, FP32).  No
// grid-wide barrier: items of all steps and phases are claimed in one
// sequence (step, phase, grid, item), and an item waits only until the
// previous phase of its own grid has completed (per-grid counters
// done[g * nph + ph] of completed items, never reset within a launch), so
// the items of other grids fill the tail of a phase.  An item
// waits only on items claimed before it, which run on resident workgroups:
// the earliest unfinished item never waits, so every wait ends.  Each item
// makes its writes visible at device scope before it counts itself done
// (one L2 write-back), and acquires once after its wait.  The wait is
// bounded; a time-out raises *err and every workgroup leaves.
template <typename T, int Q, bool FUSE>
__global__ __launch_bounds__(RX, sizeof(T) == 4 ? 2 : 1) void kb_persistent(const GridDesc<T> *d, int ng, const int *items_f,
                                                    const int *items_s, int Lf, int Ls, int nsteps, int npass,
                                                    int nlow, int bin0, unsigned *work, unsigned *done, int *err)
{
    __shared__ __attribute__((aligned(16)))
        char lds[cmax(cmax(FUSE ? 0 : front2d::front_lds_bytes<T, 0, RX>(), stream2d::stream_lds_bytes<T, 3, Q, RX>()),
                      FUSE ? cmax(fuse_lds<T, Q - 1>(), fuse_lds<T, Q>()) : 0)];
    __shared__ double sred[2 * RX / 64];
    __shared__ int s_it, sflag;
    const int nf = items_f[ng], ns = items_s[ng];
    constexpr int p0 = FUSE ? 1 : 0;
    const int nph = 1 + npass - p0;
    const unsigned per_step = (unsigned)nf + (unsigned)(npass - p0) * (unsigned)ns;
    const unsigned total = per_step * (unsigned)nsteps;
    // Control flow that the compiler sees as uniform: the claim is read back
    // with readfirstlane, and the thread-0 work that ends an item (the
    // completion count and the next claim) sits in one block followed by a
    // barrier, away from the loop's back edge.  (With the claim at the top
    // of the loop and the completion at its end, the compiler hoisted both
    // out of an inner loop that the other lanes kept running on the stale
    // claim.)
    if (threadIdx.x == 0) s_it = (int)atomicAdd(work, 1u);
    __syncthreads();
    unsigned it = (unsigned)__builtin_amdgcn_readfirstlane(s_it);
    while (it < total) {
        const int step = (int)(it / per_step);
        unsigned r = it % per_step;
        int ph, item;
        if (r < (unsigned)nf) {
            ph = 0;
            item = (int)r;
        } else {
            r -= (unsigned)nf;
            ph = 1 + (int)(r / (unsigned)ns);
            item = (int)(r % (unsigned)ns);
        }
        const int *items = ph == 0 ? items_f : items_s;
        const int g = find_grid(items, ng, item);
        if (threadIdx.x == 0) {
            // the previous phase of this grid: of this step, or the last of the previous step
            int dph = ph - 1, dstep = step;
            if (ph == 0) { dph = nph - 1; dstep = step - 1; }
            int ok = 1;
            if (dstep >= 0) {
                const int *ditems = dph == 0 ? items_f : items_s;
                const unsigned need = (unsigned)(dstep + 1) * (unsigned)(ditems[g + 1] - ditems[g]);
                const unsigned *cnt = &done[g * nph + dph];
                unsigned spins = 0;
                while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    __builtin_amdgcn_s_sleep(2);
                    // 2^21 polls: over 0.1 s of sleep alone (2 x 64 cycles per poll)
                    // plus two device-scope loads each, against an item's sub-ms run
                    if (++spins > (1u << 21) ||
                        __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            sflag = ok;
        }
        __syncthreads();
        if (!__builtin_amdgcn_readfirstlane(sflag)) return;
        const int bin = bin0 ^ (step & 1);
        if (ph == 0) {
            if constexpr (FUSE) {
                if constexpr (fuse_k<T, Q - 1>()) {
                    if (nlow > 0) front_sweep_item<T, Q - 1>(d, ng, items_f, Lf, bin, item, lds);
                }
                if constexpr (fuse_k<T, Q>()) {
                    if (nlow == 0) front_sweep_item<T, Q>(d, ng, items_f, Lf, bin, item, lds);
                }
            } else {
                front_item<T>(d, ng, items_f, Lf, bin, item, lds, sred);
            }
        } else {
            const int p = ph - 1 + p0;
            const bool first = p == 0, last = p == npass - 1;
            const int xin = (p + 1) & 1, xout = p & 1;
            bool handled = false;
            if constexpr (Q > 1) {
                if (p < nlow) {
                    if (last) sweep_item<T, Q - 1, stream2d::OM_LAST>(d, ng, items_s, Ls, first, xin, xout, item, lds, sred);
                    else sweep_item<T, Q - 1, stream2d::OM_STORE>(d, ng, items_s, Ls, first, xin, xout, item, lds, sred);
                    handled = true;
                }
            }
            if (!handled) {
                if (last) sweep_item<T, Q, stream2d::OM_LAST>(d, ng, items_s, Ls, first, xin, xout, item, lds, sred);
                else sweep_item<T, Q, stream2d::OM_STORE>(d, ng, items_s, Ls, first, xin, xout, item, lds, sred);
            }
        }
        // this item's writes are visible at device scope before it counts;
        // then the next claim
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(&done[g * nph + ph], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_it = (int)atomicAdd(work, 1u);
        }
        __syncthreads();
        it = (unsigned)__builtin_amdgcn_readfirstlane(s_it);
    }
}

template <typename T>
__global__ void kb_zero(unsigned *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// launchers (instantiated per element type in kbatch_f32.hip, kbatch_f64.hip)
// ---------------------------------------------------------------------------

template <typename T>
hipError_t launch_front_impl(const GridDesc<T> *d, int ng, const int *items, int nitems, int L, int bin,
                             hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL((kb_front<T>), dim3(nitems), dim3(RX), 0, s, d, ng, items, L, bin);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_front_sweep_impl(const GridDesc<T> *d, int ng, const int *items, int nitems, int L, int k, int bin,
                                   hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    if constexpr (sizeof(T) != 4) {
        return hipErrorInvalidValue;
    } else {
        switch (k) {
        case 3: hipLaunchKernelGGL((kb_front_sweep<T, 3>), dim3(nitems), dim3(RX), 0, s, d, ng, items, L, bin); break;
        case 4: hipLaunchKernelGGL((kb_front_sweep<T, 4>), dim3(nitems), dim3(RX), 0, s, d, ng, items, L, bin); break;
        case 5: hipLaunchKernelGGL((kb_front_sweep<T, 5>), dim3(nitems), dim3(RX), 0, s, d, ng, items, L, bin); break;
        case 6: hipLaunchKernelGGL((kb_front_sweep<T, 6>), dim3(nitems), dim3(RX), 0, s, d, ng, items, L, bin); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
}

template <typename T, int K>
hipError_t sweep_disp(const GridDesc<T> *d, int ng, const int *items, int nitems, int L, int k, bool first,
                      bool last, int xin, int xout, hipStream_t s)
{
    if constexpr (K == 0) {
        return hipErrorInvalidValue;
    } else {
        if (k != K) return sweep_disp<T, K - 1>(d, ng, items, nitems, L, k, first, last, xin, xout, s);
        if (last)
            hipLaunchKernelGGL((kb_sweep<T, K, stream2d::OM_LAST>), dim3(nitems), dim3(RX), 0, s, d, ng, items, L,
                               (int)first, xin, xout);
        else
            hipLaunchKernelGGL((kb_sweep<T, K, stream2d::OM_STORE>), dim3(nitems), dim3(RX), 0, s, d, ng, items, L,
                               (int)first, xin, xout);
        return hipGetLastError();
    }
}

template <typename T>
hipError_t launch_sweep_impl(const GridDesc<T> *d, int ng, const int *items, int nitems, int L, int k, bool first,
                             bool last, int xin, int xout, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    return sweep_disp<T, KMAX>(d, ng, items, nitems, L, k, first, last, xin, xout, s);
}

template <typename T, int Q>
int occ_q()
{
    static std::atomic<int> resident[MX_MAX_DEVICES];
    return per_device(resident, [] {
        int o = 0, o2 = 0, dev = 0, cu = 0;
        (void)hipGetDevice(&dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, kb_persistent<T, Q, false>, RX, 0) != hipSuccess) o = 0;
        if constexpr (fuse_q<T, Q>()) {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o2, kb_persistent<T, Q, true>, RX, 0) != hipSuccess) o2 = 0;
            o = std::min(o, o2);
        }
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cu = 0;
        return o * cu;
    });
}

template <typename T, int Q>
int persistent_blocks_disp(int q)
{
    if constexpr (Q == 0) {
        return 0;
    } else {
        if (q == Q) return occ_q<T, Q>();
        return persistent_blocks_disp<T, Q - 1>(q);
    }
}

// cnt[0]: the claim counter, cnt[1 .. ndone]: per-grid phase counters
template <typename T, int Q>
hipError_t persist_disp(const GridDesc<T> *d, int ng, const int *items_f, const int *items_s, int Lf, int Ls,
                     int nsteps, int q, int npass, int nlow, int bin0, unsigned *cnt, int ndone, int *err,
                     int fuse, hipStream_t s)
{
    if constexpr (Q == 0) {
        return hipErrorInvalidValue;
    } else {
        if (q != Q)
            return persist_disp<T, Q - 1>(d, ng, items_f, items_s, Lf, Ls, nsteps, q, npass, nlow, bin0, cnt, ndone,
                                       err, fuse, s);
        const int nblocks = occ_q<T, Q>();
        if (nblocks <= 0) return hipErrorInvalidValue;
        // counters start at zero (a fill kernel: no memset node in a captured stream)
        hipLaunchKernelGGL(kb_zero<T>, dim3((ndone + 1 + 255) / 256), dim3(256), 0, s, cnt, ndone + 1);
        unsigned *work = cnt, *done = cnt + 1;
        void *args[] = {(void *)&d, (void *)&ng, (void *)&items_f, (void *)&items_s, (void *)&Lf, (void *)&Ls,
                        (void *)&nsteps, (void *)&npass, (void *)&nlow, (void *)&bin0, (void *)&work, (void *)&done,
                        (void *)&err};
        if constexpr (fuse_q<T, Q>()) {
            if (fuse)
                return hipLaunchCooperativeKernel((const void *)kb_persistent<T, Q, true>, dim3(nblocks), dim3(RX), args, 0, s);
        }
        if (fuse) return hipErrorInvalidValue;
        return hipLaunchCooperativeKernel((const void *)kb_persistent<T, Q, false>, dim3(nblocks), dim3(RX), args, 0, s);
    }
}

}  // namespace batch2d
}  // namespace mx
