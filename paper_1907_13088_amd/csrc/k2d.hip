// 2D kernels of the field step: the fused front pass (current filter,
// Faraday update, auxiliary increment) and the temporally blocked
// mass-matrix sweep pass, plus the pointwise E increment and the
// deterministic FP64 reduction of per-workgroup partial sums.
//
// Equations (arXiv 1907.13088):
//   Faraday, 2D ............ eqs faraday_x_2d and the two following (Sec. 2.2.2)
//   auxiliary increment .... eqs following faraday, ending ampere_aux_z_2d
//   A, 2D .................. eqs matrixA_1st_2d .. matrixA_last_2d
//   sweeps ................. Alg 1
// The current filter is p passes of the binomial (1,2,1)/4 along x and y,
// applied here as one (2p+1)-tap binomial per axis (identical operator).
#include "mx_internal.h"

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

template <int P>
__device__ __forceinline__ constexpr float binom_w(int t)
{
    // C(2P, t) / 4^P
    float c = 1.0f;
    for (int i = 0; i < t; i++) c = c * (float)(2 * P - i) / (float)(i + 1);
    float d = 1.0f;
    for (int i = 0; i < P; i++) d *= 4.0f;
    return c / d;
}

// ---------------------------------------------------------------------------
// Front pass.  Tile of FX x FY cells; the workgroup stages E with a halo of
// one (two cells upstream), forms B^{n+1/2} on the tile plus a one-cell
// ring, filters the current in LDS, and writes B^{n+1/2} and dE'.
// B is read from B_in and written to B_out (distinct buffers), so that halo
// reads never see a neighbour tile's update.
// ---------------------------------------------------------------------------
constexpr int FX = 64, FY = 16;

template <typename T, int BLK, int P>
__global__ __launch_bounds__(NT) void k2_front(Coef<T> c, FrontArgs<T> a, const T *Bin0,
                                               const T *Bin1, const T *Bin2)
{
    constexpr bool TE = BLK & 1, TM = BLK & 2;
    constexpr int EX = FX + 3, EY = FY + 3;
    constexpr int BX = FX + 2, BY = FY + 2;
    constexpr int JX = FX + 2 * P, JY = FY + 2 * P;
    __shared__ T sE[3][EY][EX];
    __shared__ T sB[3][BY][BX];
    __shared__ T sJ[JY][JX];
    __shared__ T sJx[JY][FX];
    __shared__ double sred[2 * NT / 64];

    const int nx = c.nx, ny = c.ny;
    const int x0 = blockIdx.x * FX, y0 = blockIdx.y * FY;
    const int tid = threadIdx.x;
    const T *Bin[3] = {Bin0, Bin1, Bin2};

    for (int idx = tid; idx < EX * EY; idx += NT) {
        const int ly = idx / EX, lx = idx - ly * EX;
        const size_t o = (size_t)wrapi(y0 - 1 + ly, ny) * nx + wrapi(x0 - 1 + lx, nx);
        if (TE) { sE[0][ly][lx] = a.E[0][o]; sE[1][ly][lx] = a.E[1][o]; }
        if (TM) sE[2][ly][lx] = a.E[2][o];
    }
    __syncthreads();

    // B^{n+1/2} = B^{n-1/2} - dt curl E^n on the tile and a one-cell ring
    for (int idx = tid; idx < BX * BY; idx += NT) {
        const int ly = idx / BX, lx = idx - ly * BX;
        const int gxr = x0 - 1 + lx, gyr = y0 - 1 + ly;
        const size_t o = (size_t)wrapi(gyr, ny) * nx + wrapi(gxr, nx);
        const bool own = lx >= 1 && lx <= FX && ly >= 1 && ly <= FY && gxr < nx && gyr < ny;
        if (TM) {
            const T ez = sE[2][ly][lx];
            const T bx = Bin[0][o] - c.tdy * (sE[2][ly + 1][lx] - ez);
            const T by = Bin[1][o] + c.tdx * (sE[2][ly][lx + 1] - ez);
            sB[0][ly][lx] = bx;
            sB[1][ly][lx] = by;
            if (own) { a.B[0][o] = bx; a.B[1][o] = by; }
        }
        if (TE) {
            const T bz = Bin[2][o] - (c.tdx * (sE[1][ly][lx + 1] - sE[1][ly][lx])
                                      - c.tdy * (sE[0][ly + 1][lx] - sE[0][ly][lx]));
            sB[2][ly][lx] = bz;
            if (own) a.B[2][o] = bz;
        }
    }

    // filtered current at this thread's cells: (tx, ty + 4 r)
    const int tx = tid & 63, ty = tid >> 6;
    constexpr int R = FY / 4;
    T jf[3][R];
    for (int q = 0; q < 3; q++)
        for (int r = 0; r < R; r++) jf[q][r] = T(0);
    if (a.J0[0] != nullptr) {
        for (int q = 0; q < 3; q++) {
            if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
            __syncthreads();
            for (int idx = tid; idx < JX * JY; idx += NT) {
                const int ly = idx / JX, lx = idx - ly * JX;
                sJ[ly][lx] = a.J0[q][(size_t)wrapi(y0 - P + ly, ny) * nx + wrapi(x0 - P + lx, nx)];
            }
            __syncthreads();
            for (int idx = tid; idx < JY * FX; idx += NT) {
                const int ly = idx / FX, lx = idx - ly * FX;
                T s = T(0);
#pragma unroll
                for (int t = 0; t <= 2 * P; t++) s += T(binom_w<P>(t)) * sJ[ly][lx + t];
                sJx[ly][lx] = s;
            }
            __syncthreads();
            for (int r = 0; r < R; r++) {
                const int ly = ty + 4 * r;
                T s = T(0);
#pragma unroll
                for (int t = 0; t <= 2 * P; t++) s += T(binom_w<P>(t)) * sJx[ly + t][tx];
                jf[q][r] = s;
            }
        }
    }
    __syncthreads();

    // dE' = dt curl(Lambda B^{n+1/2}) - 4 pi dt env Jf
    const T sixth = T(1.0 / 6.0);
    const T es = a.env_src;
    double nte = 0.0, ntm = 0.0;
    for (int r = 0; r < R; r++) {
        const int ly = ty + 4 * r;
        const int gx = x0 + tx, gy = y0 + ly;
        if (gx >= nx || gy >= ny) continue;
        const size_t o = (size_t)gy * nx + gx;
        const int bx = tx + 1, by = ly + 1;
        if (TE) {
            const T bz = sB[2][by][bx];
            const T dx_ = c.tdy * (bz - sB[2][by - 1][bx]) - es * jf[0][r];
            const T dy_ = -c.tdx * (bz - sB[2][by][bx - 1]) - es * jf[1][r];
            a.dEp[0][o] = dx_;
            a.dEp[1][o] = dy_;
            nte += (double)dx_ * dx_ + (double)dy_ * dy_;
        }
        if (TM) {
            T ay0, ay1, ax0, ax1;
            if (c.lumped) {
                ay0 = sB[1][by][bx]; ay1 = sB[1][by][bx - 1];
                ax0 = sB[0][by][bx]; ax1 = sB[0][by - 1][bx];
            } else {
                // alpha f = f + (f- + f+ - 2 f)/6
                ay0 = sB[1][by][bx] + (sB[1][by - 1][bx] + sB[1][by + 1][bx] - T(2) * sB[1][by][bx]) * sixth;
                ay1 = sB[1][by][bx - 1] + (sB[1][by - 1][bx - 1] + sB[1][by + 1][bx - 1] - T(2) * sB[1][by][bx - 1]) * sixth;
                ax0 = sB[0][by][bx] + (sB[0][by][bx - 1] + sB[0][by][bx + 1] - T(2) * sB[0][by][bx]) * sixth;
                ax1 = sB[0][by - 1][bx] + (sB[0][by - 1][bx - 1] + sB[0][by - 1][bx + 1] - T(2) * sB[0][by - 1][bx]) * sixth;
            }
            const T dz_ = c.tdx * (ay0 - ay1) - c.tdy * (ax0 - ax1) - es * jf[2][r];
            a.dEp[2][o] = dz_;
            ntm += (double)dz_ * dz_;
        }
    }
    if (a.partial != nullptr) {
        block_sum2(nte, ntm, sred);
        if (tid == 0) {
            const size_t wg = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
            a.partial[2 * wg] = nte;
            a.partial[2 * wg + 1] = ntm;
        }
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
                const T ax = c.cxx * (X[cc + RX] + X[cc - RX] - T(2) * X[cc])
                           + c.cxy * ((Y[cc + 1] - Y[cc]) - (Y[cc + 1 - RX] - Y[cc - RX]));
                const T ay = c.cyy * (Y[cc + 1] + Y[cc - 1] - T(2) * Y[cc])
                           + c.cxy * ((X[cc + RX] - X[cc + RX - 1]) - (X[cc] - X[cc - 1]));
                if (!DELTA) {
                    dst[cc] = own[s][0] + ax;
                    dst[NR + cc] = own[s][1] + ay;
                } else {
                    dst[cc] = ax;
                    dst[NR + cc] = ay;
                    if (interior) { own[s][0] += ax; own[s][1] += ay; }
                }
            }
            if (TM) {
                constexpr int qz = (BLK == 2) ? 0 : 2;
                const T *Z = src + qz * NR;
                const T lx0 = Z[cc + 1] + Z[cc - 1] - T(2) * Z[cc];
                const T lxp = Z[cc + RX + 1] + Z[cc + RX - 1] - T(2) * Z[cc + RX];
                const T lxm = Z[cc - RX + 1] + Z[cc - RX - 1] - T(2) * Z[cc - RX];
                const T ly0 = Z[cc + RX] + Z[cc - RX] - T(2) * Z[cc];
                const T az = c.czx * lx0 + c.czy * ly0 + c.czz * (lxp + lxm - T(2) * lx0);
                if (!DELTA) {
                    dst[qz * NR + cc] = own[s][qz] + az;
                } else {
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

__global__ __launch_bounds__(NT) void k_reduce2(const double *partial, int nwg, double *out)
{
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

template <typename T, int BLK>
hipError_t front_blk(const Coef<T> &c, int p, const FrontArgs<T> &a, const T *const Bin[3],
                     hipStream_t s, int *nwg)
{
    dim3 grid((c.nx + FX - 1) / FX, (c.ny + FY - 1) / FY);
    *nwg = grid.x * grid.y;
    switch (p) {
    case 0: hipLaunchKernelGGL((k2_front<T, BLK, 0>), grid, dim3(NT), 0, s, c, a, Bin[0], Bin[1], Bin[2]); break;
    case 1: hipLaunchKernelGGL((k2_front<T, BLK, 1>), grid, dim3(NT), 0, s, c, a, Bin[0], Bin[1], Bin[2]); break;
    case 2: hipLaunchKernelGGL((k2_front<T, BLK, 2>), grid, dim3(NT), 0, s, c, a, Bin[0], Bin[1], Bin[2]); break;
    case 3: hipLaunchKernelGGL((k2_front<T, BLK, 3>), grid, dim3(NT), 0, s, c, a, Bin[0], Bin[1], Bin[2]); break;
    case 4: hipLaunchKernelGGL((k2_front<T, BLK, 4>), grid, dim3(NT), 0, s, c, a, Bin[0], Bin[1], Bin[2]); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_front2d(const Coef<T> &c, int blocks, int filter_passes, const FrontArgs<T> &a,
                          const T *const Bin[3], hipStream_t s, int *nwg)
{
    switch (blocks) {
    case 1: return front_blk<T, 1>(c, filter_passes, a, Bin, s, nwg);
    case 2: return front_blk<T, 2>(c, filter_passes, a, Bin, s, nwg);
    case 3: return front_blk<T, 3>(c, filter_passes, a, Bin, s, nwg);
    default: return hipErrorInvalidValue;
    }
}

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

hipError_t launch_reduce2(const double *partial, int nwg, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(NT), 0, s, partial, nwg, out);
    return hipGetLastError();
}

template hipError_t launch_front2d<float>(const Coef<float> &, int, int, const FrontArgs<float> &,
                                          const float *const[3], hipStream_t, int *);
template hipError_t launch_front2d<double>(const Coef<double> &, int, int, const FrontArgs<double> &,
                                           const double *const[3], hipStream_t, int *);
template hipError_t launch_sweep2d<float>(const Coef<float> &, int, int, bool, int,
                                          const SweepArgs<float> &, hipStream_t, int *);
template hipError_t launch_sweep2d<double>(const Coef<double> &, int, int, bool, int,
                                           const SweepArgs<double> &, hipStream_t, int *);
template hipError_t launch_update<float>(int64_t, int, float *const[3], const float *const[3], hipStream_t);
template hipError_t launch_update<double>(int64_t, int, double *const[3], const double *const[3], hipStream_t);

}  // namespace mx
