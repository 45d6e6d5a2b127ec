#pragma once
// Streaming (2.5D) temporally blocked mass-matrix sweep pass for 2D grids
// (Alg 1 with A from eqs matrixA_1st_2d .. matrixA_last_2d).
//
// A workgroup owns a strip of RX columns, one column per thread, and walks
// down a chunk of rows.  Sweep level l (1..K) computes row t - 2l at time
// step t, so every input row it needs from level l-1 was produced at an
// earlier step: one barrier per step suffices.  Each thread keeps its own
// column's recent values per level in registers (sliding windows of 2-3
// rows); the only cross-thread traffic is the newest row of each level,
// exchanged through a double-buffered LDS row (5 neighbour reads per cell
// and sweep).  The valid columns shrink by one per level on each side, so a
// strip writes RX - 2K columns; rows are pipelined, so a chunk of L rows
// recomputes only K extra rows per level at each end.
//
// Standard form: x_l = b + A x_(l-1), b = dE' carried along with the row
// (slot 0 of a level's carried window holds the carried value of the row the
// level produced last; the next level reads it before the producer shifts).
// Delta form:    d_l = A d_(l-1), s_l = s_(l-1) + d_l, s carried along.
#include <algorithm>
#include <type_traits>

#include "mx_internal.h"
#include "stencil2d.h"

namespace mx {
namespace stream2d {

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

// output modes of the last level (compile time, so the steady step is one
// basic block): store the iterate, add it to E, or store it and accumulate
// the FP64 norm of the last sweep's step
enum : int { OM_STORE = 0, OM_LAST = 1, OM_RESID = 2 };

// One work item: strip wid % nsx, chunk wid / nsx of rows [Y0, Y0 + L).
// pidx is where the item's FP64 partial sums go (OM_RESID only).
// LDS a tile needs: one double-buffered row of 3 components per level
template <typename T, int K, int RX>
constexpr size_t stream_lds_bytes() { return sizeof(T) * (size_t)K * 2 * 3 * (RX + 2); }

template <typename T, int BLK, int K, bool DELTA, int RX, int OM>
__device__ __forceinline__ void stream_tile(const Coef<T> &c, const SweepArgs<T> &a, int flags, int L, int nsx,
                                            int wid, int pidx, void *lds, double *sred)
{
    constexpr bool TE = BLK & 1, TM = BLK & 2;
    constexpr int W = RX - 2 * K;
    constexpr int PAD = RX + 2;
    T(*xs)[2][3][PAD] = reinterpret_cast<T(*)[2][3][PAD]>(lds);

    const int sx = wid % nsx, sy = wid / nsx;

    const int nx = c.nx, ny = c.ny;
    const int i = threadIdx.x;
    const int X0 = sx * W, Y0 = sy * L;
    const int gxi = X0 - K + i;
    const int gx = wrapi(gxi, nx);
    const bool first = flags & SW_FIRST;
    constexpr bool last = OM == OM_LAST;
    constexpr bool resid = OM == OM_RESID;
    constexpr bool store = OM != OM_LAST;
    const bool outcol = i >= K && i < RX - K && gxi < nx;

    T out[K + 1][3];
    T wex[K + 1][3], wez[K + 1][3], wg[K + 1][3], wlx[K + 1][3];
    T wley[K + 1][2], wh[K + 1][2], wey[K + 1][2];
    T wc[K + 1][2][3];
#pragma unroll
    for (int l = 0; l <= K; l++)
#pragma unroll
        for (int q = 0; q < 3; q++) {
            out[l][q] = wex[l][q] = wez[l][q] = wg[l][q] = wlx[l][q] = T(0);
            wc[l][0][q] = wc[l][1][q] = T(0);
            if (q < 2) wley[l][q] = wh[l][q] = wey[l][q] = T(0);
        }

    // rows are prefetched two steps ahead into two register sets (by parity)
    T px[2][3], pc[2][3], pe[2][3];
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
        for (int q = 0; q < 3; q++) px[u][q] = pc[u][q] = pe[u][q] = T(0);
    // uniform bases of the level-0 iterate and of the carried quantity (on the
    // first pass both are dE': the second read of a row hits the cache)
    const T *xb[3], *cb[3];
#pragma unroll
    for (int q = 0; q < 3; q++) {
        xb[q] = first ? a.rhs[q] : a.x_in[q];
        cb[q] = (DELTA && !first) ? a.s_in[q] : a.rhs[q];
    }
    auto load_row = [&](int row, T(&x)[3], T(&cc)[3]) {
        const unsigned o = (unsigned)(wrapi(row, ny) * nx + gx) * (unsigned)sizeof(T);
#pragma unroll
        for (int q = 0; q < 3; q++) {
            if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
            x[q] = ld_off(xb[q], o);
            cc[q] = ld_off(cb[q], o);
        }
    };
    auto load_e = [&](int row, T(&e)[3]) {
        if (!(last && outcol && row >= Y0 && row < Y0 + L && row < ny)) return;
        const unsigned o = (unsigned)(row * nx + gxi) * (unsigned)sizeof(T);
#pragma unroll
        for (int q = 0; q < 3; q++) {
            if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
            e[q] = ld_off(a.E[q], o);
        }
    };

    const int tbeg = Y0 - K, tend = Y0 + L + 2 * K;
    // E row r is added at step r + 2K (parity of r), x row t at step t
    load_row(tbeg, px[tbeg & 1], pc[tbeg & 1]);
    load_row(tbeg + 1, px[(tbeg + 1) & 1], pc[(tbeg + 1) & 1]);
    load_e(tbeg - 2 * K, pe[tbeg & 1]);
    load_e(tbeg + 1 - 2 * K, pe[(tbeg + 1) & 1]);
    double rte = 0.0, rtm = 0.0;

    // One time step.  ALL: every level receives and computes (the steady
    // state between pipeline fill and drain), so no row-range tests are needed
    // and the window shifts become register renaming once unrolled.
    auto step = [&](const int t, auto all_tag, auto par_tag) {
        constexpr bool ALL = decltype(all_tag)::value;
        // parity of t: compile time in the unrolled steady state (t even at
        // the start of each group), so LDS slot addresses are constants there
        const int pw = ALL ? decltype(par_tag)::value : (t & 1);
        const int pr = pw ^ 1;
#pragma unroll
        for (int l = K; l >= 1; l--) {
            // arrival of row t-2l+1 of level l-1 (computed at the previous step)
            const int rho = t - 2 * l + 1;
            if (ALL || (rho >= Y0 - K + (l - 1) && rho < Y0 + L + K - (l - 1))) {
                const T *X = &xs[l - 1][pr][0][0];
                const T *Y = &xs[l - 1][pr][1][0];
                const T *Z = &xs[l - 1][pr][2][0];
                if (TE) {
                    const T exn = out[l - 1][0], eyn = out[l - 1][1];
                    const T eyp = Y[i + 2], eym = Y[i], exm = X[i];
                    wex[l][0] = wex[l][1]; wex[l][1] = wex[l][2]; wex[l][2] = exn;
                    wg[l][0] = wg[l][1]; wg[l][1] = wg[l][2]; wg[l][2] = eyp - eyn;
                    wley[l][0] = wley[l][1]; wley[l][1] = d2(eym, eyn, eyp);
                    wh[l][0] = wh[l][1]; wh[l][1] = exn - exm;
                    wey[l][0] = wey[l][1]; wey[l][1] = eyn;
                }
                if (TM) {
                    const T ezn = out[l - 1][2];
                    const T ezp = Z[i + 2], ezm = Z[i];
                    wez[l][0] = wez[l][1]; wez[l][1] = wez[l][2]; wez[l][2] = ezn;
                    wlx[l][0] = wlx[l][1]; wlx[l][1] = wlx[l][2]; wlx[l][2] = d2(ezm, ezn, ezp);
                }
#pragma unroll
                for (int q = 0; q < 3; q++) { wc[l][0][q] = wc[l][1][q]; wc[l][1][q] = wc[l - 1][0][q]; }
            }
            // row t-2l of level l
            const int r = t - 2 * l;
            if (ALL || (r >= Y0 - K + l && r < Y0 + L + K - l)) {
                T nv[3] = {T(0), T(0), T(0)}, nc[3] = {T(0), T(0), T(0)};
                if (TE) {
                    const T ax = a_te_x(c.cxx, c.cxy, d2(wex[l][0], wex[l][1], wex[l][2]), wg[l][1] - wg[l][0]);
                    const T ay = a_te_y(c.cyy, c.cxy, wley[l][0], wh[l][1] - wh[l][0]);
                    if (!DELTA) {
                        nv[0] = wc[l][0][0] + ax; nv[1] = wc[l][0][1] + ay;
                        nc[0] = wc[l][0][0]; nc[1] = wc[l][0][1];
                    } else {
                        nv[0] = ax; nv[1] = ay;
                        nc[0] = wc[l][0][0] + ax; nc[1] = wc[l][0][1] + ay;
                    }
                }
                if (TM) {
                    const T lx0 = wlx[l][1];
                    const T ly0 = d2(wez[l][0], wez[l][1], wez[l][2]);
                    const T az = a_tm(c.czx, c.czy, c.czz, lx0, ly0, d2(wlx[l][0], lx0, wlx[l][2]));
                    if (!DELTA) { nv[2] = wc[l][0][2] + az; nc[2] = wc[l][0][2]; }
                    else { nv[2] = az; nc[2] = wc[l][0][2] + az; }
                }
                if (l < K) {
#pragma unroll
                    for (int q = 0; q < 3; q++) {
                        if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
                        out[l][q] = nv[q];
                        wc[l][0][q] = nc[q];   // carried value of this row, read by level l+1 next step
                        xs[l][pw][q][i + 1] = nv[q];
                    }
                } else if (outcol && r >= Y0 && r < ny) {
                    const unsigned o = (unsigned)(r * nx + gxi) * (unsigned)sizeof(T);
                    if (resid) {
                        if (TE) {
                            const double d0 = DELTA ? (double)nv[0] : (double)nv[0] - (double)wex[l][1];
                            const double d1 = DELTA ? (double)nv[1] : (double)nv[1] - (double)wey[l][0];
                            rte += d0 * d0 + d1 * d1;
                        }
                        if (TM) {
                            const double d2 = DELTA ? (double)nv[2] : (double)nv[2] - (double)wez[l][1];
                            rtm += d2 * d2;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < 3; q++) {
                        if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
                        if (store) {
                            st_off(a.x_out[q], o, nv[q]);
                            if (DELTA) st_off(a.s_out[q], o, nc[q]);
                        }
                        if (last) st_off(a.E[q], o, pe[pw][q] + (DELTA ? nc[q] : nv[q]));
                    }
                }
            }
        }
        // level 0: the row loaded for this step
        if (ALL || t < Y0 + L + K) {
#pragma unroll
            for (int q = 0; q < 3; q++) {
                if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
                out[0][q] = px[pw][q];
                wc[0][0][q] = pc[pw][q];
                xs[0][pw][q][i + 1] = px[pw][q];
            }
            // the freed set receives row t+2 (in the unrolled body
            // unconditionally: a row past the end is a valid, unused row)
            if (ALL || t + 2 < Y0 + L + K) load_row(t + 2, px[pw], pc[pw]);
        }
        load_e(t + 2 - 2 * K, pe[pw]);
        lds_barrier();
    };

    // fill, steady state (every level active), drain
    const int ts0 = Y0 + 2 * K, ts1 = Y0 + L + K;
    int t = tbeg;
    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    for (; (t < ts0 || (t & 1)) && t < tend; t++) step(t, std::false_type{}, P0{});
    constexpr int U = 6;   // multiple of the window periods (2 and 3) and even
    for (; t + U <= ts1; t += U) {
        step(t + 0, std::true_type{}, P0{});
        step(t + 1, std::true_type{}, P1{});
        step(t + 2, std::true_type{}, P0{});
        step(t + 3, std::true_type{}, P1{});
        step(t + 4, std::true_type{}, P0{});
        step(t + 5, std::true_type{}, P1{});
    }
    for (; t < tend; t++) step(t, std::false_type{}, P0{});
    if (resid) {
        block_sum2<RX>(rte, rtm, sred);
        if (threadIdx.x == 0) {
            a.partial[2 * pidx] = rte;
            a.partial[2 * pidx + 1] = rtm;
        }
    }
    lds_barrier();   // the LDS rows are reused by the caller's next item
}

// work item of a single-grid launch: consecutive chunks of a strip go to the
// same XCD (workgroups are dealt round-robin over the 8 XCDs)
__device__ __forceinline__ int xcd_item(int nwg)
{
    const int b = blockIdx.x;
    const int per = (nwg + 7) / 8;
    const int wid = (b % 8) * per + b / 8;
    return (nwg % 8 != 0 || wid >= nwg) ? b : wid;
}

template <typename T, int BLK, int K, bool DELTA, int RX, int OM>
__global__ __launch_bounds__(RX) void k2_stream(Coef<T> c, SweepArgs<T> a, int flags, int L, int nsx, int nwg)
{
    __shared__ __attribute__((aligned(16))) char lds[stream_lds_bytes<T, K, RX>()];
    __shared__ double sred[2 * RX / 64];
    stream_tile<T, BLK, K, DELTA, RX, OM>(c, a, flags, L, nsx, xcd_item(nwg), blockIdx.x, lds, sred);
}

constexpr int SRX = 256;

template <typename T, int BLK, int K, bool DELTA, int OM>
hipError_t stream_om(const Coef<T> &c, int flags, const SweepArgs<T> &a, hipStream_t s, int *nwg, int slots)
{
    constexpr int W = SRX - 2 * K;
    static int occ = -1, ncu = -1;
    if (occ < 0) {
        int o = 0, dev = 0, cu = 0;
        (void)hipGetDevice(&dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k2_stream<T, BLK, K, DELTA, SRX, OM>, SRX, 0) != hipSuccess || o < 1) o = 1;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu < 1) cu = 256;
        ncu = cu;
        occ = o;
    }
    if (slots <= 0) slots = occ * ncu;
    const int nsx = (c.nx + W - 1) / W;
    // one resident round: choose the chunk count so that strips x chunks fill
    // the resident workgroup slots, then round the chunk length up
    int nsy = std::max(1, slots / nsx);
    nsy = std::min(nsy, c.ny);
    int L = (c.ny + nsy - 1) / nsy;
    L = std::max(L, std::min(c.ny, 4 * K));   // bound the pipeline fill overhead
    nsy = (c.ny + L - 1) / L;
    const int n = nsx * nsy;
    *nwg = n;
    hipLaunchKernelGGL((k2_stream<T, BLK, K, DELTA, SRX, OM>), dim3(n), dim3(SRX), 0, s, c, a, flags, L, nsx, n);
    return hipGetLastError();
}

template <typename T, int BLK, int K, bool DELTA>
hipError_t stream_k(const Coef<T> &c, int flags, const SweepArgs<T> &a, hipStream_t s, int *nwg, int slots)
{
    const int out = flags & (SW_LAST | SW_STORE | SW_RESID);
    if (out == SW_LAST) return stream_om<T, BLK, K, DELTA, OM_LAST>(c, flags, a, s, nwg, slots);
    if (out == SW_STORE) return stream_om<T, BLK, K, DELTA, OM_STORE>(c, flags, a, s, nwg, slots);
    if (out == (SW_STORE | SW_RESID)) return stream_om<T, BLK, K, DELTA, OM_RESID>(c, flags, a, s, nwg, slots);
    return hipErrorInvalidValue;
}

template <typename T, int BLK, bool DELTA>
hipError_t stream_blk(const Coef<T> &c, int k, int flags, const SweepArgs<T> &a, hipStream_t s, int *nwg,
                      int slots)
{
    switch (k) {
    case 1: return stream_k<T, BLK, 1, DELTA>(c, flags, a, s, nwg, slots);
    case 2: return stream_k<T, BLK, 2, DELTA>(c, flags, a, s, nwg, slots);
    case 3: return stream_k<T, BLK, 3, DELTA>(c, flags, a, s, nwg, slots);
    case 4: return stream_k<T, BLK, 4, DELTA>(c, flags, a, s, nwg, slots);
    case 5: return stream_k<T, BLK, 5, DELTA>(c, flags, a, s, nwg, slots);
    case 6: return stream_k<T, BLK, 6, DELTA>(c, flags, a, s, nwg, slots);
    case 7: return stream_k<T, BLK, 7, DELTA>(c, flags, a, s, nwg, slots);
    case 8: return stream_k<T, BLK, 8, DELTA>(c, flags, a, s, nwg, slots);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, bool DELTA>
hipError_t launch(const Coef<T> &c, int blocks, int k, int flags, const SweepArgs<T> &a, hipStream_t s,
                  int *nwg, int slots)
{
    switch (blocks) {
    case 1: return stream_blk<T, 1, DELTA>(c, k, flags, a, s, nwg, slots);
    case 2: return stream_blk<T, 2, DELTA>(c, k, flags, a, s, nwg, slots);
    case 3: return stream_blk<T, 3, DELTA>(c, k, flags, a, s, nwg, slots);
    }
    return hipErrorInvalidValue;
}

}  // namespace stream2d
}  // namespace mx
