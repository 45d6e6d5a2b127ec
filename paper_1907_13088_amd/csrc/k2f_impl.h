#pragma once
// Streaming front pass of the 2D field step (arXiv 1907.13088, Sec. 2.2.2):
//   Faraday update of B (eqs faraday_x_2d and following),
//   low-pass filter of the current (p binomial (1,2,1)/4 passes per axis),
//   auxiliary increment dE' = dt curl(Lambda B^{n+1/2}) - 4 pi dt env Jf
//   (the 2D auxiliary equations ending with ampere_aux_z_2d).
//
// A workgroup owns a strip of RX columns (one per thread) and walks down a
// chunk of rows.  At step t it receives row t of E and of the old B, forms
// B^{n+1/2} of row t-1, completes the x-neighbour terms of B^{n+1/2} row t-2,
// and emits dE' of row t-3.  The current row t+p-2 is filtered along x by a
// (2p+1)-tap binomial over an LDS row and along y by p cascaded 3-tap passes
// in two-row register windows, so the filtered row t-3 is ready at the same
// step (the x and y filters commute, so this equals p alternating passes).
// Neighbour columns go through double-buffered LDS rows: one barrier per
// step.  Columns within max(p,1) (left) and max(p,2) (right) of the strip
// edges are halo; the strip writes the rest.
#include <algorithm>
#include <type_traits>

#include "mx_internal.h"

namespace mx {
namespace front2d {

__device__ __forceinline__ int wrapi(int i, int n)
{
    if (i >= 0 && i < n) return i;
    int r = i % n;
    return r < 0 ? r + n : r;
}

template <int NTH>
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
        for (int q = 0; q < NTH / 64; q++) { a += sh[2 * q]; b += sh[2 * q + 1]; }
    }
}

template <int P>
__device__ __forceinline__ constexpr float binom(int t)
{
    float c = 1.0f;
    for (int i = 0; i < t; i++) c = c * (float)(2 * P - i) / (float)(i + 1);
    float d = 1.0f;
    for (int i = 0; i < P; i++) d *= 4.0f;
    return c / d;
}

// alpha f = f + (f- + f+ - 2 f)/6 (the 1-4-1 average of Sec. 2, written so
// that a constant passes through exactly)
template <typename T>
__device__ __forceinline__ T avg6(T fm, T f0, T fp, T sixth)
{
    // sixth = 1/6, or 0 for the lumped (Yee) scheme: then exactly f0
    return fma(fma(T(-2), f0, fm + fp), sixth, f0);
}

// LDS a tile needs: double-buffered rows of E (2 components), B and J (3 each)
template <typename T, int P, int RX>
constexpr size_t front_lds_bytes() { return sizeof(T) * (size_t)2 * 8 * (RX + 2 * (P > 1 ? P : 1)); }

template <typename T, int BLK, int P, int RX, bool HASJ>
__device__ __forceinline__ void front_tile(const Coef<T> &c, const FrontArgs<T> &a, const T *Bin0,
                                           const T *Bin1, const T *Bin2, int L, int nsx, int wid, int pidx,
                                           void *lds, double *sred)
{
    constexpr bool TE = BLK & 1, TM = BLK & 2;
    constexpr int HL = front_aligned() ? 16 : (P > 1 ? P : 1);
    constexpr int W = front_aligned() ? RX - 32 : RX - HL - (P > 2 ? P : 2);
    static_assert(HL >= (P > 1 ? P : 1) && RX - HL - W >= (P > 2 ? P : 2), "the halo must cover the stencils");
    constexpr int PADL = P > 1 ? P : 1;
    constexpr int PR = RX + 2 * PADL;
    constexpr int D = P - 2;           // the current is loaded D rows ahead of E
    constexpr int NP = P > 0 ? P : 1;
    T(*sE)[2][PR] = reinterpret_cast<T(*)[2][PR]>(lds);                        // Ey, Ez of the newest E row
    T(*sB)[3][PR] = reinterpret_cast<T(*)[3][PR]>((T *)lds + 2 * 2 * PR);      // newest B^{n+1/2} row
    T(*sJ)[3][PR] = reinterpret_cast<T(*)[3][PR]>((T *)lds + 2 * 5 * PR);      // newest raw current row

    const int sx = wid % nsx, sy = wid / nsx;

    const int nx = c.nx, ny = c.ny;
    const int i = threadIdx.x;
    const int li = i + PADL;
    const int X0 = sx * W, Y0 = sy * L;
    L = std::min(L, c.ny - Y0);   // a grid's last chunk may be short: run only its rows
    const int gxi = X0 - HL + i;
    const int gx = wrapi(gxi, nx);
    const bool outcol = i >= HL && i < HL + W && gxi < nx;
    constexpr bool hasj = HASJ;   // a prescribed current is present (a.J0 non-null)
    const T sixth = c.lumped ? T(0) : T(1.0 / 6.0);
    const T es = a.env_src;

    // rows are prefetched two steps ahead into two register sets (by parity)
    T pE[2][3], pB[2][3], pJ[2][3];
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
        for (int q = 0; q < 3; q++) pE[u][q] = pB[u][q] = pJ[u][q] = T(0);
    T e1[3] = {T(0), T(0), T(0)};      // own E, row t-1
    T bo1[3] = {T(0), T(0), T(0)};     // own old B, row t-1
    T bp1[3] = {T(0), T(0), T(0)};     // own B^{n+1/2}, row t-2
    // windows for dE' of row r = t-3 (newest entry is row r+1 = t-2)
    T by_w[3] = {T(0), T(0), T(0)};    // own By, rows r-1, r, r+1
    T byl_w[3] = {T(0), T(0), T(0)};   // By of column i-1
    T axbx_w[3] = {T(0), T(0), T(0)};  // alpha_x Bx (own column)
    T bz_w[3] = {T(0), T(0), T(0)};    // own Bz
    T dxbz_w[2] = {T(0), T(0)};        // Bz(i) - Bz(i-1), rows r, r+1
    T fy[NP][3][2];                    // y-filter cascade windows
#pragma unroll
    for (int k = 0; k < NP; k++)
#pragma unroll
        for (int q = 0; q < 3; q++) fy[k][q][0] = fy[k][q][1] = T(0);

    // rows are loaded in order, one per step: byte offsets of the next E/B
    // row and of the next current row advance with a wrap (uniform scalars)
    const int tb = std::min(Y0 - 1, Y0 - 2 * P + 2), te = Y0 + L + 3;
    const unsigned rowb = (unsigned)nx * (unsigned)sizeof(T);
    const unsigned allb = rowb * (unsigned)ny;
    const unsigned colb = (unsigned)gx * (unsigned)sizeof(T);
    unsigned loe = (unsigned)wrapi(tb, ny) * rowb, loj = (unsigned)wrapi(tb + D, ny) * rowb;
    auto load = [&](T(&e)[3], T(&bb)[3], T(&j)[3]) {
        const unsigned oe = loe + colb;
#pragma unroll
        for (int q = 0; q < 3; q++) {
            if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
            e[q] = ld_off(a.E[q], oe);
        }
        if (TM) { bb[0] = ld_off(Bin0, oe); bb[1] = ld_off(Bin1, oe); }
        if (TE) bb[2] = ld_off(Bin2, oe);
        loe += rowb;
        if (loe >= allb) loe -= allb;
        if constexpr (hasj) {
            const unsigned oj = loj + colb;
#pragma unroll
            for (int q = 0; q < 3; q++) {
                if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
                j[q] = ld_off(a.J0[q], oj);
            }
            loj += rowb;
            if (loj >= allb) loj -= allb;
        }
    };

    load(pE[tb & 1], pB[tb & 1], pJ[tb & 1]);
    if (tb + 1 < te) load(pE[(tb + 1) & 1], pB[(tb + 1) & 1], pJ[(tb + 1) & 1]);
    double nte = 0.0, ntm = 0.0;

    auto step = [&](const int t, auto par_tag, auto all_tag) {
        constexpr bool ALL = decltype(all_tag)::value;
        const int pw = ALL ? decltype(par_tag)::value : (t & 1);
        const int pr = pw ^ 1;
        const T e0[3] = {pE[pw][0], pE[pw][1], pE[pw][2]};
        const T bo0[3] = {pB[pw][0], pB[pw][1], pB[pw][2]};
        const T jr[3] = {pJ[pw][0], pJ[pw][1], pJ[pw][2]};
        // the freed register set receives row t+2 (in the unrolled body
        // unconditionally: a row past the end is a valid, unused row)
        if (ALL || t + 2 < te) load(pE[pw], pB[pw], pJ[pw]);
        // B^{n+1/2} of row t-1 = B^{n-1/2} - dt curl E^n (E rows t-1 and t)
        T bp0[3] = {T(0), T(0), T(0)};
        if (TM) {
            const T ezr = sE[pr][1][li + 1];
            bp0[0] = bo1[0] - c.tdy * (e0[2] - e1[2]);
            bp0[1] = bo1[1] + c.tdx * (ezr - e1[2]);
        }
        if (TE) {
            const T eyr = sE[pr][0][li + 1];
            bp0[2] = bo1[2] - (c.tdx * (eyr - e1[1]) - c.tdy * (e0[0] - e1[0]));
        }
        // x-neighbour terms of B^{n+1/2} row t-2 (formed at the previous step)
        if (TM) {
            const T bxl = sB[pr][0][li - 1], bxr = sB[pr][0][li + 1];
            axbx_w[0] = axbx_w[1]; axbx_w[1] = axbx_w[2]; axbx_w[2] = avg6(bxl, bp1[0], bxr, sixth);
            byl_w[0] = byl_w[1]; byl_w[1] = byl_w[2]; byl_w[2] = sB[pr][1][li - 1];
            by_w[0] = by_w[1]; by_w[1] = by_w[2]; by_w[2] = bp1[1];
        }
        if (TE) {
            dxbz_w[0] = dxbz_w[1]; dxbz_w[1] = bp1[2] - sB[pr][2][li - 1];
            bz_w[0] = bz_w[1]; bz_w[1] = bz_w[2]; bz_w[2] = bp1[2];
        }
        // current: x filter of row t-1+D, then p cascaded y passes -> row t-3
        T jf[3] = {T(0), T(0), T(0)};
        if constexpr (hasj) {
#pragma unroll
            for (int q = 0; q < 3; q++) {
                if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
                T v = T(0);
#pragma unroll
                for (int k = -P; k <= P; k++) v = fma(T(binom<P>(k + P)), sJ[pr][q][li + k], v);
#pragma unroll
                for (int k = 0; k < P; k++) {
                    const T o = T(0.25) * fma(T(2), fy[k][q][1], fy[k][q][0] + v);
                    fy[k][q][0] = fy[k][q][1];
                    fy[k][q][1] = v;
                    v = o;
                }
                jf[q] = v;
            }
        }
        // dE' of row r = t-3
        const int r = t - 3;
        if (outcol && r >= Y0 && r < Y0 + L && r < ny) {
            const unsigned o = (unsigned)(r * nx + gxi) * (unsigned)sizeof(T);
            if (TE) {
                const T vx = c.tdy * (bz_w[1] - bz_w[0]) - es * jf[0];
                const T vy = -c.tdx * dxbz_w[0] - es * jf[1];
                st_off(a.dEp[0], o, vx);
                st_off(a.dEp[1], o, vy);
                if (a.partial) nte += (double)vx * vx + (double)vy * vy;
            }
            if (TM) {
                const T ay = avg6(by_w[0], by_w[1], by_w[2], sixth);
                const T ayl = avg6(byl_w[0], byl_w[1], byl_w[2], sixth);
                const T vz = c.tdx * (ay - ayl) - c.tdy * (axbx_w[1] - axbx_w[0]) - es * jf[2];
                st_off(a.dEp[2], o, vz);
                if (a.partial) ntm += (double)vz * vz;
            }
        }
        // publish row t of E, B^{n+1/2} row t-1 and current row t+D
        if (TE) sE[pw][0][li] = e0[1];
        if (TM) sE[pw][1][li] = e0[2];
        // B components of a block: TE owns Bz, TM owns Bx and By
        if (TM) { sB[pw][0][li] = bp0[0]; sB[pw][1][li] = bp0[1]; }
        if (TE) sB[pw][2][li] = bp0[2];
        if constexpr (hasj) {
            // the current is placed like E: TE owns Jx, Jy; TM owns Jz
            if (TE) { sJ[pw][0][li] = jr[0]; sJ[pw][1][li] = jr[1]; }
            if (TM) sJ[pw][2][li] = jr[2];
        }
        const int rb = t - 1;
        if (outcol && rb >= Y0 && rb < Y0 + L && rb < ny) {
            const unsigned o = (unsigned)(rb * nx + gxi) * (unsigned)sizeof(T);
            if (TM) { st_off(a.B[0], o, bp0[0]); st_off(a.B[1], o, bp0[1]); }
            if (TE) st_off(a.B[2], o, bp0[2]);
        }
#pragma unroll
        for (int q = 0; q < 3; q++) { e1[q] = e0[q]; bo1[q] = bo0[q]; bp1[q] = bp0[q]; }
        lds_barrier();
    };

    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    int t = tb;
    for (; (t & 1) && t < te; t++) step(t, P0{}, std::false_type{});
    for (; t + 6 <= te; t += 6) {
        step(t + 0, P0{}, std::true_type{});
        step(t + 1, P1{}, std::true_type{});
        step(t + 2, P0{}, std::true_type{});
        step(t + 3, P1{}, std::true_type{});
        step(t + 4, P0{}, std::true_type{});
        step(t + 5, P1{}, std::true_type{});
    }
    for (; t < te; t++) step(t, P0{}, std::false_type{});

    if (a.partial != nullptr) {
        block_sum2<RX>(nte, ntm, sred);
        if (threadIdx.x == 0) {
            a.partial[2 * pidx] = nte;
            a.partial[2 * pidx + 1] = ntm;
        }
    }
    lds_barrier();   // the LDS rows are reused by the caller's next item
}

template <typename T, int BLK, int P, int RX, bool HASJ>
__global__ __launch_bounds__(RX) void k2_front_stream(Coef<T> c, FrontArgs<T> a, const T *Bin0,
                                                      const T *Bin1, const T *Bin2, int L, int nsx, int nwg)
{
    const int b = blockIdx.x;
    const int wid = xcd_map(blockIdx.x, nwg);
    __shared__ __attribute__((aligned(16))) char lds[front_lds_bytes<T, P, RX>()];
    __shared__ double sred[2 * RX / 64];
    front_tile<T, BLK, P, RX, HASJ>(c, a, Bin0, Bin1, Bin2, L, nsx, wid, b, lds, sred);
}

}  // namespace front2d
}  // namespace mx
