// Batched stepping of independent 2D periodic grids (each with its own size,
// time step and coefficients; no current; a fixed number m of sweeps).
//
// Every grid is cut into work items exactly as a single-grid launch would
// cut it (strips of columns x chunks of rows), and the items of all grids
// are concatenated: item it belongs to grid g with items[g] <= it <
// items[g+1].  Two schedules:
//  * grouped: one launch per phase (front, then each sweep pass) covering
//    the items of every grid;
//  * persistent: one cooperative launch runs all steps; workgroups claim the
//    items of each phase from an atomic counter (so uneven items balance)
//    and meet at a grid-wide barrier between phases.  The barrier's wait is
//    bounded: on time-out it raises an error flag and every workgroup
//    leaves, so the launch always drains.
#pragma once

#include "gridbar.h"
#include "k2f_impl.h"
#include "k2s_impl.h"

namespace mx {
namespace batch2d {

constexpr int RX = STRIP;

// largest g with items[g] <= it, items[0] = 0, items[ng] = total
__device__ __forceinline__ int find_grid(const int *items, int ng, int it)
{
    int lo = 0, hi = ng;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (items[mid] <= it) lo = mid; else hi = mid;
    }
    return lo;
}

template <typename T>
__device__ __forceinline__ void front_item(const GridDesc<T> *d, int ng, const int *items, int L, int bin, int it,
                                           void *lds, double *sred)
{
    const int g = find_grid(items, ng, it);
    const GridDesc<T> &gd = d[g];
    FrontArgs<T> fa;
    for (int q = 0; q < 3; q++) {
        fa.E[q] = gd.E[q];
        fa.B[q] = gd.B[bin ^ 1][q];
        fa.J0[q] = nullptr;
        fa.dEp[q] = gd.dEp[q];
    }
    fa.env_src = T(0);
    fa.partial = nullptr;
    front2d::front_tile<T, 3, 0, RX, false>(gd.c, fa, gd.B[bin][0], gd.B[bin][1], gd.B[bin][2], L, gd.nsx_f,
                                            it - items[g], 0, lds, sred);
}

template <typename T, int K, int OM>
__device__ __forceinline__ void sweep_item(const GridDesc<T> *d, int ng, const int *items, int L, bool first,
                                           int xin, int xout, int it, void *lds, double *sred)
{
    const int g = find_grid(items, ng, it);
    const GridDesc<T> &gd = d[g];
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
    stream2d::stream_tile<T, 3, K, false, RX, OM>(gd.c, sa, first ? SW_FIRST : 0, L, gd.nsx_s, it - items[g], 0,
                                                  lds, sred);
}

template <typename T>
__global__ __launch_bounds__(RX) void kb_front(const GridDesc<T> *d, int ng, const int *items, int L, int bin)
{
    __shared__ __attribute__((aligned(16))) char lds[front2d::front_lds_bytes<T, 0, RX>()];
    __shared__ double sred[2 * RX / 64];
    front_item<T>(d, ng, items, L, bin, xcd_map(blockIdx.x, gridDim.x), lds, sred);
}

template <typename T, int K, int OM>
__global__ __launch_bounds__(RX) void kb_sweep(const GridDesc<T> *d, int ng, const int *items, int L, int first,
                                               int xin, int xout)
{
    __shared__ __attribute__((aligned(16))) char lds[stream2d::stream_lds_bytes<T, 3, K, RX>()];
    __shared__ double sred[2 * RX / 64];
    sweep_item<T, K, OM>(d, ng, items, L, first != 0, xin, xout, xcd_map(blockIdx.x, gridDim.x), lds, sred);
}

// Claim items [0, n) one at a time from the phase's work counter.
template <typename F>
__device__ __forceinline__ void claim_items(unsigned *work, int n, int *s_it, F &&f)
{
    for (;;) {
        if (threadIdx.x == 0) *s_it = (int)atomicAdd(work, 1u);
        __syncthreads();
        const int it = *s_it;
        __syncthreads();   // every thread has read the claim before the next one
        if (it >= n) break;
        f(it);
    }
}

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }

// All nsteps steps of all grids in one launch; npass passes per step, the
// first nlow of Q - 1 sweeps, the others of Q.
template <typename T, int Q>
__global__ __launch_bounds__(RX, sizeof(T) == 4 ? 2 : 1) void kb_persistent(const GridDesc<T> *d, int ng, const int *items_f,
                                                    const int *items_s, int Lf, int Ls, int nsteps, int npass,
                                                    int nlow, int bin0, unsigned *bar, int *err)
{
    __shared__ __attribute__((aligned(16)))
        char lds[cmax(front2d::front_lds_bytes<T, 0, RX>(), stream2d::stream_lds_bytes<T, 3, Q, RX>())];
    __shared__ double sred[2 * RX / 64];
    __shared__ int sflag, s_it;
    const int nf = items_f[ng], ns = items_s[ng];
    unsigned *work = &bar[2];
    int bin = bin0;
    for (int step = 0; step < nsteps; step++) {
        claim_items(work, nf, &s_it, [&](int it) { front_item<T>(d, ng, items_f, Lf, bin, it, lds, sred); });
        bin ^= 1;
        if (!grid_barrier(bar, gridDim.x, err, &sflag)) return;
        for (int p = 0; p < npass; p++) {
            const bool first = p == 0, last = p == npass - 1;
            const int xin = (p + 1) & 1, xout = p & 1;
            const bool low = p < nlow;
            claim_items(work, ns, &s_it, [&](int it) {
                if constexpr (Q > 1) {
                    if (low) {
                        if (last)
                            sweep_item<T, Q - 1, stream2d::OM_LAST>(d, ng, items_s, Ls, first, xin, xout, it, lds,
                                                                    sred);
                        else
                            sweep_item<T, Q - 1, stream2d::OM_STORE>(d, ng, items_s, Ls, first, xin, xout, it, lds,
                                                                     sred);
                        return;
                    }
                }
                if (last) sweep_item<T, Q, stream2d::OM_LAST>(d, ng, items_s, Ls, first, xin, xout, it, lds, sred);
                else sweep_item<T, Q, stream2d::OM_STORE>(d, ng, items_s, Ls, first, xin, xout, it, lds, sred);
            });
            if (!grid_barrier(bar, gridDim.x, err, &sflag)) return;
        }
    }
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
        int o = 0, dev = 0, cu = 0;
        (void)hipGetDevice(&dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, kb_persistent<T, Q>, RX, 0) != hipSuccess) o = 0;
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

template <typename T, int Q>
hipError_t persist_disp(const GridDesc<T> *d, int ng, const int *items_f, const int *items_s, int Lf, int Ls,
                        int nsteps, int q, int npass, int nlow, int bin0, unsigned *bar, int *err, int nblocks,
                        hipStream_t s)
{
    if constexpr (Q == 0) {
        return hipErrorInvalidValue;
    } else {
        if (q != Q)
            return persist_disp<T, Q - 1>(d, ng, items_f, items_s, Lf, Ls, nsteps, q, npass, nlow, bin0, bar, err,
                                          nblocks, s);
        void *args[] = {(void *)&d, (void *)&ng, (void *)&items_f, (void *)&items_s, (void *)&Lf, (void *)&Ls,
                        (void *)&nsteps, (void *)&npass, (void *)&nlow, (void *)&bin0, (void *)&bar, (void *)&err};
        return hipLaunchCooperativeKernel((const void *)kb_persistent<T, Q>, dim3(nblocks), dim3(RX), args, 0, s);
    }
}

}  // namespace batch2d
}  // namespace mx
