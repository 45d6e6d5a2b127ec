// Batched stepping of independent 2D periodic grids (each with its own size,
// time step and coefficients; no current; a fixed number m of sweeps).
//
// Every grid is cut into work items exactly as a single-grid launch would
// cut it (strips of columns x chunks of rows), and the items of all grids
// are concatenated: item it belongs to grid g with items[g] <= it <
// items[g+1].  Two schedules:
//  * grouped: one launch per phase (front, then each sweep pass) covering
//    the items of every grid;
//  * persistent: one cooperative launch runs all steps; workgroups stride
//    over the items of each phase and meet at a grid-wide barrier between
//    phases.  The barrier's wait is bounded: on time-out it raises an error
//    flag and every workgroup leaves, so the launch always drains.
#pragma once

#include "k2f_impl.h"
#include "k2s_impl.h"

namespace mx {
namespace batch2d {

constexpr int RX = 256;

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
    stream2d::stream_tile<T, 3, K, false, RX, OM>(gd.c, sa, first ? SW_FIRST : 0, L, gd.nsx_s, it - items[g], 0,
                                                  lds, sred);
}

template <typename T>
__global__ __launch_bounds__(RX) void kb_front(const GridDesc<T> *d, int ng, const int *items, int L, int bin)
{
    __shared__ __attribute__((aligned(16))) char lds[front2d::front_lds_bytes<T, 0, RX>()];
    __shared__ double sred[2 * RX / 64];
    front_item<T>(d, ng, items, L, bin, blockIdx.x, lds, sred);
}

template <typename T, int K, int OM>
__global__ __launch_bounds__(RX) void kb_sweep(const GridDesc<T> *d, int ng, const int *items, int L, int first,
                                               int xin, int xout)
{
    __shared__ __attribute__((aligned(16))) char lds[stream2d::stream_lds_bytes<T, 3, K, RX>()];
    __shared__ double sred[2 * RX / 64];
    sweep_item<T, K, OM>(d, ng, items, L, first != 0, xin, xout, blockIdx.x, lds, sred);
}

// Grid-wide barrier for a cooperative launch.  All threads fence their
// global writes at device scope (other XCDs' L2s must see them), thread 0
// arrives on a counter and waits for the generation to move; the wait is
// bounded.  Returns false (every thread) after a time-out.
__device__ __forceinline__ bool grid_barrier(unsigned *bar, unsigned nblocks, int *err, int *sflag)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned prev = atomicAdd(&bar[0], 1u);
        if (prev == nblocks - 1) {
            atomicExch(&bar[0], 0u);
            __threadfence();
            atomicAdd(&bar[1], 1u);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1u << 25)) {   // about two seconds
                    atomicOr(err, 1);
                    ok = 0;
                    break;
                }
            }
        }
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
        *sflag = ok;
    }
    __syncthreads();
    const bool ok = *sflag != 0;
    __threadfence();
    return ok;
}

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }

// All nsteps steps of all grids in one launch; passes of exactly Q sweeps
// (m = npass * Q).
template <typename T, int Q>
__global__ __launch_bounds__(RX) void kb_persistent(const GridDesc<T> *d, int ng, const int *items_f,
                                                    const int *items_s, int Lf, int Ls, int nsteps, int npass,
                                                    int bin0, unsigned *bar, int *err)
{
    __shared__ __attribute__((aligned(16)))
        char lds[cmax(front2d::front_lds_bytes<T, 0, RX>(), stream2d::stream_lds_bytes<T, 3, Q, RX>())];
    __shared__ double sred[2 * RX / 64];
    __shared__ int sflag;
    const int nf = items_f[ng], ns = items_s[ng];
    int bin = bin0;
    for (int step = 0; step < nsteps; step++) {
        for (int it = blockIdx.x; it < nf; it += gridDim.x) front_item<T>(d, ng, items_f, Lf, bin, it, lds, sred);
        bin ^= 1;
        if (!grid_barrier(bar, gridDim.x, err, &sflag)) return;
        for (int p = 0; p < npass; p++) {
            const bool first = p == 0, last = p == npass - 1;
            const int xin = (p + 1) & 1, xout = p & 1;
            for (int it = blockIdx.x; it < ns; it += gridDim.x) {
                if (last) sweep_item<T, Q, stream2d::OM_LAST>(d, ng, items_s, Ls, first, xin, xout, it, lds, sred);
                else sweep_item<T, Q, stream2d::OM_STORE>(d, ng, items_s, Ls, first, xin, xout, it, lds, sred);
            }
            if (!grid_barrier(bar, gridDim.x, err, &sflag)) return;
        }
    }
}

}  // namespace batch2d
}  // namespace mx
