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
#include "mx_internal.h"
#include "stencil2d.h"

namespace mx {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ int wrapi(int i, int n)
{
    if (i >= 0 && i < n) return i;
    int r = i % n;
    return r < 0 ? r + n : r;
}

template <int BLK> struct NComp;
template <> struct NComp<1> { static constexpr int n = 2; };   // TE: Ex, Ey
template <> struct NComp<2> { static constexpr int n = 1; };   // TM: Ez
template <> struct NComp<3> { static constexpr int n = 3; };

// global component of local slot q
template <int BLK>
__device__ __forceinline__ constexpr int gq(int q) { return BLK == 2 ? 2 : q; }

// Sum two doubles over the workgroup in a fixed order; valid in thread 0.
__device__ void block_sum2(double &a, double &b, double *sh)
{
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) { sh[2 * w] = a; sh[2 * w + 1] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = 0.0; b = 0.0;
        for (int i = 0; i < NT / 64; i++) { a += sh[2 * i]; b += sh[2 * i + 1]; }
    }
}

// ---------------------------------------------------------------------------
// Sweep pass: K fused sweeps x <- b + A x (standard form) or d <- A d,
// s <- s + d (delta form) on an LDS region of (TX + 2K) x (TY + 2K) cells
// whose valid part shrinks by one cell per side per sweep; the TX x TY
// interior is written back once.  Ping-pong LDS buffers, one barrier per
// sweep.
// ---------------------------------------------------------------------------
template <typename T, int BLK, int K, int TX, int TY, bool DELTA>
__global__ __launch_bounds__(NT) void k2_sweep(Coef<T> c, SweepArgs<T> a, int flags)
{
    if (a.skip && *a.skip) return;   // the block has met its stop test
    constexpr int NC = NComp<BLK>::n;
    constexpr int RX = TX + 2 * K, RY = TY + 2 * K, NR = RX * RY;
    constexpr int NS = (NR + NT - 1) / NT;
    constexpr bool TE = BLK & 1, TM = BLK & 2;
    __shared__ T buf[2][NC][NR];
    __shared__ double sred[2 * NT / 64];

    const int nx = c.nx, ny = c.ny;
    const int rx0 = blockIdx.x * TX - K, ry0 = blockIdx.y * TY - K;
    const int tid = threadIdx.x;
    const bool first = flags & SW_FIRST;

    T own[NS][NC];   // b (standard) at every owned cell; s (delta) at owned interior cells
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const int cc = tid + NT * s;
        if (cc >= NR) break;
        const int cy = cc / RX, cx = cc - cy * RX;
        const size_t o = (size_t)wrapi(ry0 + cy, ny) * nx + wrapi(rx0 + cx, nx);
        const bool interior = cx >= K && cx < K + TX && cy >= K && cy < K + TY;
#pragma unroll
        for (int q = 0; q < NC; q++) {
            const int g = gq<BLK>(q);
            const T xin = first ? a.rhs[g][o] : a.x_in[g][o];
            buf[0][q][cc] = xin;
            if (!DELTA) own[s][q] = first ? xin : a.rhs[g][o];
            else own[s][q] = interior ? (first ? xin : a.s_in[g][o]) : T(0);
        }
    }
    __syncthreads();

#pragma unroll
    for (int l = 1; l <= K; l++) {
        const T *src = &buf[(l - 1) & 1][0][0];
        T *dst = &buf[l & 1][0][0];
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const int cc = tid + NT * s;
            if (cc >= NR) break;
            const int cy = cc / RX, cx = cc - cy * RX;
            if (cx < l || cx >= RX - l || cy < l || cy >= RY - l) continue;
            const bool interior = cx >= K && cx < K + TX && cy >= K && cy < K + TY;
            if (TE) {
                const T *X = src, *Y = src + NR;
                const T lyy = d2(X[cc - RX], X[cc], X[cc + RX]);
                const T dg = (Y[cc + 1] - Y[cc]) - (Y[cc + 1 - RX] - Y[cc - RX]);
                const T lxx = d2(Y[cc - 1], Y[cc], Y[cc + 1]);
                const T dh = (X[cc + RX] - X[cc + RX - 1]) - (X[cc] - X[cc - 1]);
                if (!DELTA) {
                    dst[cc] = a_te_x_b(c.cxx, c.cxy, lyy, dg, own[s][0]);
                    dst[NR + cc] = a_te_y_b(c.cyy, c.cxy, lxx, dh, own[s][1]);
                } else {
                    const T ax = a_te_x(c.cxx, c.cxy, lyy, dg);
                    const T ay = a_te_y(c.cyy, c.cxy, lxx, dh);
                    dst[cc] = ax;
                    dst[NR + cc] = ay;
                    if (interior) { own[s][0] += ax; own[s][1] += ay; }
                }
            }
            if (TM) {
                constexpr int qz = (BLK == 2) ? 0 : 2;
                const T *Z = src + qz * NR;
                const T lx0 = d2(Z[cc - 1], Z[cc], Z[cc + 1]);
                const T lxp = d2(Z[cc + RX - 1], Z[cc + RX], Z[cc + RX + 1]);
                const T lxm = d2(Z[cc - RX - 1], Z[cc - RX], Z[cc - RX + 1]);
                const T ly0 = d2(Z[cc - RX], Z[cc], Z[cc + RX]);
                if (!DELTA) {
                    dst[qz * NR + cc] = a_tm_b(c.czx, c.czy, c.czz, lx0, ly0, d2(lxm, lx0, lxp), own[s][qz]);
                } else {
                    const T az = a_tm(c.czx, c.czy, c.czz, lx0, ly0, d2(lxm, lx0, lxp));
                    dst[qz * NR + cc] = az;
                    if (interior) own[s][qz] += az;
                }
            }
        }
        __syncthreads();
    }

    const T *fin = &buf[K & 1][0][0];
    const T *prv = &buf[(K - 1) & 1][0][0];
    double rte = 0.0, rtm = 0.0;
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const int cc = tid + NT * s;
        if (cc >= NR) break;
        const int cy = cc / RX, cx = cc - cy * RX;
        if (cx < K || cx >= K + TX || cy < K || cy >= K + TY) continue;
        const int gx = rx0 + cx, gy = ry0 + cy;
        if (gx >= nx || gy >= ny) continue;
        const size_t o = (size_t)gy * nx + gx;
#pragma unroll
        for (int q = 0; q < NC; q++) {
            const int g = gq<BLK>(q);
            const T v = fin[q * NR + cc];
            if (flags & SW_RESID) {
                const double d = DELTA ? (double)v : (double)v - (double)prv[q * NR + cc];
                if (g == 2) rtm += d * d; else rte += d * d;
            }
            if (flags & SW_STORE) {
                a.x_out[g][o] = v;
                if (DELTA) a.s_out[g][o] = own[s][q];
            }
            if (flags & SW_LAST) a.E[g][o] += DELTA ? own[s][q] : v;
        }
    }
    if (flags & SW_RESID) {
        block_sum2(rte, rtm, sred);
        if (tid == 0) {
            const size_t wg = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
            a.partial[2 * wg] = rte;
            a.partial[2 * wg + 1] = rtm;
        }
    }
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
