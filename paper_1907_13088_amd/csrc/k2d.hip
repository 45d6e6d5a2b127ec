// 2D kernels of the field step: the LDS-tile temporally blocked mass-matrix
// sweep pass, the pointwise E increment and the deterministic FP64 reduction
// of per-workgroup partial sums.  (The front pass is in k2f.hip, the
// row-streaming sweep pass in k2s*.)
//
// Equations (arXiv 1907.13088):
//   Faraday, 2D ............ eqs faraday_x_2d and the two following (Sec. 2.2.2)
//   auxiliary increment .... eqs following faraday, ending ampere_aux_z_2d
//   A, 2D .................. eqs matrixA_1st_2d .. matrixA_last_2d
//   sweeps ................. Alg 1
// The current filter is p passes of the binomial (1,2,1)/4 along x and y,
// applied here as one (2p+1)-tap binomial per axis (identical operator).
#include "k2tile.h"

namespace mx {
namespace {

using tile2d::NT;

template <typename T, int BLK, int K, int TX, int TY, bool DELTA>
__global__ __launch_bounds__(NT) void k2_sweep(Coef<T> c, SweepArgs<T> a, int flags)
{
    if (a.skip && *a.skip) return;   // the block has met its stop test
    __shared__ __attribute__((aligned(16))) char lds[tile2d::sweep_lds_bytes<T, BLK, K, TX, TY>()];
    __shared__ double sred[2 * NT / 64];
    tile2d::sweep_tile<T, BLK, K, TX, TY, DELTA>(c, a, flags, blockIdx.x, blockIdx.y,
                                                (size_t)blockIdx.y * gridDim.x + blockIdx.x, lds, sred);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_update(int64_t n, int mask, T *E0, T *E1, T *E2,
                                               const T *X0, const T *X1, const T *X2)
{
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    if (mask & 1) E0[i] += X0[i];
    if (mask & 2) E1[i] += X1[i];
    if (mask & 4) E2[i] += X2[i];
}

__global__ __launch_bounds__(NT) void k_reduce2(const double *partial, int nwg, double *out, const int *skip)
{
    if (skip && *skip) return;   // the pass whose partials these are did not run
    __shared__ double sa[NT], sb[NT];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nwg; i += NT) { a += partial[2 * i]; b += partial[2 * i + 1]; }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) { sa[threadIdx.x] += sa[threadIdx.x + w]; sb[threadIdx.x] += sb[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = sa[0]; out[1] = sb[0]; }
}

// tile shape of the sweep pass per element type
template <typename T> struct SweepTile { static constexpr int TX = 64, TY = 16; };
template <> struct SweepTile<double> { static constexpr int TX = 64, TY = 8; };

template <typename T, int BLK, int K, bool DELTA>
hipError_t sweep_k(const Coef<T> &c, int flags, const SweepArgs<T> &a, hipStream_t s, int *nwg)
{
    constexpr int TX = SweepTile<T>::TX, TY = SweepTile<T>::TY;
    dim3 grid((c.nx + TX - 1) / TX, (c.ny + TY - 1) / TY);
    *nwg = grid.x * grid.y;
    hipLaunchKernelGGL((k2_sweep<T, BLK, K, TX, TY, DELTA>), grid, dim3(NT), 0, s, c, a, flags);
    return hipGetLastError();
}

template <typename T, int BLK, bool DELTA>
hipError_t sweep_blk(const Coef<T> &c, int k, int flags, const SweepArgs<T> &a, hipStream_t s, int *nwg)
{
    switch (k) {
    case 1: return sweep_k<T, BLK, 1, DELTA>(c, flags, a, s, nwg);
    case 2: return sweep_k<T, BLK, 2, DELTA>(c, flags, a, s, nwg);
    case 3: return sweep_k<T, BLK, 3, DELTA>(c, flags, a, s, nwg);
    case 4: return sweep_k<T, BLK, 4, DELTA>(c, flags, a, s, nwg);
    case 5: return sweep_k<T, BLK, 5, DELTA>(c, flags, a, s, nwg);
    case 6: return sweep_k<T, BLK, 6, DELTA>(c, flags, a, s, nwg);
    case 7: return sweep_k<T, BLK, 7, DELTA>(c, flags, a, s, nwg);
    case 8: return sweep_k<T, BLK, 8, DELTA>(c, flags, a, s, nwg);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <typename T>
hipError_t launch_sweep2d(const Coef<T> &c, int blocks, int k, bool delta, int flags,
                          const SweepArgs<T> &a, hipStream_t s, int *nwg)
{
    if (delta) {
        switch (blocks) {
        case 1: return sweep_blk<T, 1, true>(c, k, flags, a, s, nwg);
        case 2: return sweep_blk<T, 2, true>(c, k, flags, a, s, nwg);
        case 3: return sweep_blk<T, 3, true>(c, k, flags, a, s, nwg);
        }
    } else {
        switch (blocks) {
        case 1: return sweep_blk<T, 1, false>(c, k, flags, a, s, nwg);
        case 2: return sweep_blk<T, 2, false>(c, k, flags, a, s, nwg);
        case 3: return sweep_blk<T, 3, false>(c, k, flags, a, s, nwg);
        }
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_update(int64_t n, int mask, T *const E[3], const T *const X[3], hipStream_t s)
{
    const int64_t nb = (n + NT - 1) / NT;
    hipLaunchKernelGGL((k_update<T>), dim3((unsigned)nb), dim3(NT), 0, s, n, mask, E[0], E[1], E[2],
                       X[0], X[1], X[2]);
    return hipGetLastError();
}

hipError_t launch_reduce2(const double *partial, int nwg, double *out, hipStream_t s, const int *skip)
{
    hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(NT), 0, s, partial, nwg, out, skip);
    return hipGetLastError();
}

__global__ void k_tol_init(TolState *st, const double *red, int nblk)
{
    if (threadIdx.x != 0) return;
    int bad = 0;
    for (int b = 0; b < 2; b++) {
        const double r = b < nblk ? sqrt(red[b]) : 0.0;
        const bool fin = isfinite(r);
        if (!fin) bad = 1;
        st->rhsn[b] = r;
        st->resid[b] = 0.0;
        st->skip[b] = (r == 0.0 || !fin) ? 1 : 0;   // dE' = 0: the increment is 0, no sweeps
        st->done[b] = 0;
        st->conv[b] = 0;
        st->last[b] = -1;
    }
    st->nonfinite = bad;
    st->pad = 0;
}

__global__ void k_tol_decide(TolState *st, const double *red, int b, int k, int buf, double tol)
{
    if (threadIdx.x != 0 || st->skip[b]) return;   // the pass did not run
    st->done[b] += k;
    st->last[b] = buf;
    const double r = sqrt(red[b]);
    st->resid[b] = r;
    if (!isfinite(r)) {
        st->nonfinite |= 2;
        st->skip[b] = 1;
    } else if (r <= tol * st->rhsn[b]) {
        st->conv[b] = 1;
        st->skip[b] = 1;
    }
}

hipError_t launch_tol_init(TolState *st, const double *red, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(k_tol_init, dim3(1), dim3(64), 0, s, st, red, nblk);
    return hipGetLastError();
}

hipError_t launch_tol_decide(TolState *st, const double *red, int b, int k, int buf, double tol, hipStream_t s)
{
    hipLaunchKernelGGL(k_tol_decide, dim3(1), dim3(64), 0, s, st, red, b, k, buf, tol);
    return hipGetLastError();
}

template hipError_t launch_sweep2d<float>(const Coef<float> &, int, int, bool, int,
                                          const SweepArgs<float> &, hipStream_t, int *);
template hipError_t launch_sweep2d<double>(const Coef<double> &, int, int, bool, int,
                                           const SweepArgs<double> &, hipStream_t, int *);
template hipError_t launch_update<float>(int64_t, int, float *const[3], const float *const[3], hipStream_t);
template hipError_t launch_update<double>(int64_t, int, double *const[3], const double *const[3], hipStream_t);

}  // namespace mx
