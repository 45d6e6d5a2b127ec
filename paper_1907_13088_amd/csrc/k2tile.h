#pragma once
// The LDS-tile sweep pass of the 2D mass-matrix solve (Alg. 1, A from eqs
// matrixA_1st_2d .. matrixA_last_2d) as a device function on one tile, so
// that the per-launch kernel and the single-launch small-grid solve run the
// same per-cell arithmetic (bitwise equal iterates).
#include "mx_internal.h"
#include "stencil2d.h"

namespace mx {
namespace tile2d {

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

// Sum two doubles over a workgroup of NTH threads in a fixed order; valid in
// thread 0.
template <int NTH = NT>
__device__ __forceinline__ void block_sum2(double &a, double &b, double *sh)
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
        for (int i = 0; i < NTH / 64; i++) { a += sh[2 * i]; b += sh[2 * i + 1]; }
    }
}

// LDS bytes of a tile pass of K sweeps
template <typename T, int BLK, int K, int TX, int TY>
constexpr size_t sweep_lds_bytes() { return sizeof(T) * 2 * NComp<BLK>::n * (TX + 2 * K) * (TY + 2 * K); }

// ---------------------------------------------------------------------------
// Sweep pass: K fused sweeps x <- b + A x (standard form) or d <- A d,
// s <- s + d (delta form) on an LDS region of (TX + 2K) x (TY + 2K) cells
// whose valid part shrinks by one cell per side per sweep; the TX x TY
// interior is written back once.  Ping-pong LDS buffers, one barrier per
// sweep.
// ---------------------------------------------------------------------------
// Tile (bx, by) of TX x TY output cells, NTH threads; `lds` holds
// sweep_lds_bytes bytes; the FP64 partial norms (TE, TM) of the last sweep
// go to partial[2 wg].  RUNTIME: the pass runs `levels` <= K sweeps in a
// level loop that is not unrolled (one code path for every pass depth, on
// the region of K; each cell's arithmetic is that of a pass of `levels`).
template <typename T, int BLK, int K, int TX, int TY, bool DELTA, int NTH = NT, bool RUNTIME = false>
__device__ __forceinline__ void sweep_tile(const Coef<T> &c, const SweepArgs<T> &a, int flags, int bx, int by,
                                           size_t wg, void *lds, double *sred, int levels = K)
{
    const int KL = RUNTIME ? levels : K;
    constexpr int NC = NComp<BLK>::n;
    constexpr int RX = TX + 2 * K, RY = TY + 2 * K, NR = RX * RY;
    constexpr int NS = (NR + NTH - 1) / NTH;
    constexpr bool TE = BLK & 1, TM = BLK & 2;
    T(*buf)[NC][NR] = reinterpret_cast<T(*)[NC][NR]>(lds);

    const int nx = c.nx, ny = c.ny;
    const int rx0 = bx * TX - K, ry0 = by * TY - K;
    const int tid = threadIdx.x;
    const bool first = flags & SW_FIRST;

    T own[NS][NC];   // b (standard) at every owned cell; s (delta) at owned interior cells
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const int cc = tid + NTH * s;
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

#pragma unroll(RUNTIME ? 1 : K)
    for (int l = 1; l <= KL; l++) {
        const T *src = &buf[(l - 1) & 1][0][0];
        T *dst = &buf[l & 1][0][0];
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const int cc = tid + NTH * s;
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

    const T *fin = &buf[KL & 1][0][0];
    const T *prv = &buf[(KL - 1) & 1][0][0];
    double rte = 0.0, rtm = 0.0;
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const int cc = tid + NTH * s;
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
        block_sum2<NTH>(rte, rtm, sred);
        if (tid == 0) {
            a.partial[2 * wg] = rte;
            a.partial[2 * wg + 1] = rtm;
        }
    }
}

}  // namespace tile2d
}  // namespace mx

