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
// Chebyshev form: r = b + A x_(l-1) - x_(l-1), d_l = f_l d_(l-1) + g_l r,
// x_l = x_(l-1) + d_l, with b and d carried along (f, g per sweep and block).
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

// LDS rows: TE levels hold (Ex, Ey) pairs (one 8- or 16-byte write and one
// paired read per cell), TM levels hold Ez
template <typename T>
struct alignas(2 * sizeof(T)) Pair {
    T x, y;
};

// rows in flight per thread (prefetch depth), a divisor of 6; three or six
// rows measured no faster than two
template <typename T, int BLK, int K>
constexpr int stream_pf() { return 2; }

// both blocks: one 16- or 32-byte record per column, (Ey, Ez) first so that
// the right neighbour's pair is one aligned 8- or 16-byte read
template <typename T>
struct alignas(4 * sizeof(T)) Quad {
    T ey, ez, ex, pad;
};
template <typename T>
struct alignas(4 * sizeof(T)) Triple {
    T ey, ez, ex;
};

// LDS words per column and level: TE 2, TM 1, both 4 (a padded record)
constexpr int stream_nc(int blk) { return blk == 3 ? 4 : blk == 1 ? 2 : 1; }

// LDS a tile needs: one double-buffered row of each carried component per level
template <typename T, int BLK, int K, int RX>
constexpr size_t stream_lds_bytes() { return sizeof(T) * (size_t)K * 2 * stream_nc(BLK) * (RX + 2); }

// One work item: strip wid % nsx, chunk wid / nsx of rows [Y0, Y0 + L).
// pidx is where the item's FP64 partial sums go (OM_RESID only).
template <typename T, int BLK, int K, int FORM, int RX, int OM>
__device__ __forceinline__ void stream_tile(const Coef<T> &c, const SweepArgs<T> &a, int flags, int L, int nsx,
                                            int wid, int pidx, void *lds, double *sred)
{
    constexpr bool TE = BLK & 1, TM = BLK & 2;
    constexpr bool DELTA = FORM == FM_DELTA, CHEB = FORM == FM_CHEB;
    constexpr int H = stream_halo(K);          // columns left of the first output column
    constexpr int W = stream_width<RX>(K);
    static_assert(H >= K && RX - H - W >= K, "the halo must cover every level");
    constexpr int PAD = RX + 2;
    // column j of a level row sits at index j + 1 - (strip origin - K)
    constexpr bool BOTH = TE && TM;
    Pair<T>(*xp)[2][PAD] = reinterpret_cast<Pair<T>(*)[2][PAD]>(lds);     // TE only
    T(*xz)[2][PAD] = reinterpret_cast<T(*)[2][PAD]>(lds);                 // TM only
    Quad<T>(*xq)[2][PAD] = reinterpret_cast<Quad<T>(*)[2][PAD]>(lds);     // both

    const int sx = wid % nsx, sy = wid / nsx;

    const int nx = c.nx, ny = c.ny;
    const int i = threadIdx.x;
    const int X0 = sx * W, Y0 = sy * L;
    L = std::min(L, c.ny - Y0);   // a grid's last chunk may be short: run only its rows
    const int gxi = X0 - H + i;
    const int gx = wrapi(gxi, nx);
    const bool first = flags & SW_FIRST;
    constexpr bool last = OM == OM_LAST;
    constexpr bool resid = OM == OM_RESID;
    constexpr bool store = OM != OM_LAST;
    const bool outcol = i >= H && i < H + W && gxi < nx;
    const int rend = std::min(Y0 + L, ny);   // rows this item writes: [Y0, rend)

    T out[K + 1][3];
    T wex[K + 1][3], wez[K + 1][3], wg[K + 1][3], wlx[K + 1][3];
    T wley[K + 1][2], wh[K + 1][2], wey[K + 1][2];
    T wc[K + 1][2][3];
    T wd[K + 1][2][3];   // Chebyshev form: the carried increment, like wc
#pragma unroll
    for (int l = 0; l <= K; l++)
#pragma unroll
        for (int q = 0; q < 3; q++) {
            out[l][q] = wex[l][q] = wez[l][q] = wg[l][q] = wlx[l][q] = T(0);
            wc[l][0][q] = wc[l][1][q] = T(0);
            wd[l][0][q] = wd[l][1][q] = T(0);
            if (q < 2) wley[l][q] = wh[l][q] = wey[l][q] = T(0);
        }

    // rows are prefetched PF steps ahead through a FIFO of PF register sets
    // (in the unrolled steady state the shifts are register renaming)
    constexpr int PF = stream_pf<T, BLK, K>();
    static_assert(6 % PF == 0, "the unrolled group of 6 steps must cycle the FIFO");
    T px[PF][3], pc[PF][3], pe[PF][3], pd[PF][3];
#pragma unroll
    for (int u = 0; u < PF; u++)
#pragma unroll
        for (int q = 0; q < 3; q++) px[u][q] = pc[u][q] = pe[u][q] = pd[u][q] = T(0);
    // uniform bases of the level-0 iterate and of the carried quantity (on the
    // first pass both are dE': the second read of a row hits the cache)
    const T *xb[3], *cb[3];
#pragma unroll
    for (int q = 0; q < 3; q++) {
        xb[q] = first ? a.rhs[q] : a.x_in[q];
        cb[q] = (DELTA && !first) ? a.s_in[q] : a.rhs[q];
    }
    // byte offset of the next level-0 row to load, advanced with a wrap
    // (a uniform scalar), plus the thread's column
    const unsigned rowb = (unsigned)nx * (unsigned)sizeof(T);
    const unsigned allb = rowb * (unsigned)ny;
    const unsigned colb = (unsigned)gx * (unsigned)sizeof(T);
    const int tbeg = Y0 - K, tend = Y0 + L + 2 * K;
    // Every step runs in the steady form (all levels, no row-range tests) in
    // groups of 6 from the even step at or before tbeg: a level's value for a
    // row outside its range feeds only rows outside the next level's range,
    // and every store and E load tests its row.  (Steps with range tests
    // took 2.8 times the instructions of a steady step.)
    const int tstart = tbeg - (tbeg & 1);
    unsigned lo = (unsigned)wrapi(tstart, ny) * rowb;
    auto load_row = [&](T(&x)[3], T(&cc)[3], T(&dd)[3]) {
        const unsigned o = lo + colb;
#pragma unroll
        for (int q = 0; q < 3; q++) {
            if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
            x[q] = ld_off(xb[q], o);
            cc[q] = ld_off(cb[q], o);
            // Chebyshev form: the increment that produced the input iterate
            // (none before the first sweep: the values read are then unused)
            if (CHEB) dd[q] = ld_off(a.s_in[q], o);
        }
        lo += rowb;
        if (lo >= allb) lo -= allb;
    };
    auto load_e = [&](int row, T(&e)[3]) {
        if (!(last && outcol && row >= Y0 && row < rend)) return;
        const unsigned o = (unsigned)(row * nx + gxi) * (unsigned)sizeof(T);
#pragma unroll
        for (int q = 0; q < 3; q++) {
            if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
            e[q] = ld_off(a.E[q], o);
        }
    };

    // x row t is consumed at step t, E row r at step r + 2K, both from the
    // head of the FIFO
#pragma unroll
    for (int u = 0; u < PF; u++) {
        load_row(px[u], pc[u], pd[u]);
        load_e(tstart + u - 2 * K, pe[u]);
    }
    double rte = 0.0, rtm = 0.0;

    // One time step.  ALL: every level receives and computes (the steady
    // state between pipeline fill and drain), so no row-range tests are needed
    // and the window shifts become register renaming once unrolled.
    auto step = [&](const int t, auto all_tag, auto slot_tag) {
        constexpr bool ALL = decltype(all_tag)::value;
        constexpr int SL = decltype(slot_tag)::value;   // position in the group of 6 (ALL)
        constexpr int ps = 0;
        // LDS row buffer of this step: compile time in the unrolled steady
        // state, so LDS slot addresses are constants there
        const int pw = ALL ? (SL & 1) : (t & 1);
        const int pr = pw ^ 1;
#pragma unroll
        for (int l = K; l >= 1; l--) {
            // arrival of row t-2l+1 of level l-1 (computed at the previous step)
            const int rho = t - 2 * l + 1;
            if (ALL || (rho >= Y0 - K + (l - 1) && rho < Y0 + L + K - (l - 1))) {
                T exm, eym, eyp, ezm, ezp;
                if (BOTH) {
                    const Quad<T> qm = xq[l - 1][pr][i];                                   // column - 1
                    const Pair<T> qp = *reinterpret_cast<const Pair<T> *>(&xq[l - 1][pr][i + 2]);  // (Ey, Ez), column + 1
                    exm = qm.ex; eym = qm.ey; ezm = qm.ez; eyp = qp.x; ezp = qp.y;
                } else if (TE) {
                    const Pair<T> pm = xp[l - 1][pr][i];       // column - 1
                    const Pair<T> pp = xp[l - 1][pr][i + 2];   // column + 1
                    exm = pm.x; eym = pm.y; eyp = pp.y; ezm = ezp = T(0);
                } else {
                    ezp = xz[l - 1][pr][i + 2]; ezm = xz[l - 1][pr][i];
                    exm = eym = eyp = T(0);
                }
                if (TE) {
                    const T exn = out[l - 1][0], eyn = out[l - 1][1];
                    wex[l][0] = wex[l][1]; wex[l][1] = wex[l][2]; wex[l][2] = exn;
                    wg[l][0] = wg[l][1]; wg[l][1] = wg[l][2]; wg[l][2] = eyp - eyn;
                    wley[l][0] = wley[l][1]; wley[l][1] = d2(eym, eyn, eyp);
                    wh[l][0] = wh[l][1]; wh[l][1] = exn - exm;
                    wey[l][0] = wey[l][1]; wey[l][1] = eyn;
                }
                if (TM) {
                    const T ezn = out[l - 1][2];
                    wez[l][0] = wez[l][1]; wez[l][1] = wez[l][2]; wez[l][2] = ezn;
                    wlx[l][0] = wlx[l][1]; wlx[l][1] = wlx[l][2]; wlx[l][2] = d2(ezm, ezn, ezp);
                }
#pragma unroll
                for (int q = 0; q < 3; q++) { wc[l][0][q] = wc[l][1][q]; wc[l][1][q] = wc[l - 1][0][q]; }
                if (CHEB) {
#pragma unroll
                    for (int q = 0; q < 3; q++) { wd[l][0][q] = wd[l][1][q]; wd[l][1][q] = wd[l - 1][0][q]; }
                }
            }
            // row t-2l of level l
            const int r = t - 2 * l;
            if (ALL || (r >= Y0 - K + l && r < Y0 + L + K - l)) {
                T nv[3] = {T(0), T(0), T(0)}, nc[3] = {T(0), T(0), T(0)};
                if (TE) {
                    const T lyy = d2(wex[l][0], wex[l][1], wex[l][2]);
                    const T dg = wg[l][1] - wg[l][0];
                    const T dh = wh[l][1] - wh[l][0];
                    if (!DELTA) {
                        nv[0] = a_te_x_b(c.cxx, c.cxy, lyy, dg, wc[l][0][0]);
                        nv[1] = a_te_y_b(c.cyy, c.cxy, wley[l][0], dh, wc[l][0][1]);
                        nc[0] = wc[l][0][0]; nc[1] = wc[l][0][1];
                    } else {
                        nv[0] = a_te_x(c.cxx, c.cxy, lyy, dg);
                        nv[1] = a_te_y(c.cyy, c.cxy, wley[l][0], dh);
                        nc[0] = wc[l][0][0] + nv[0]; nc[1] = wc[l][0][1] + nv[1];
                    }
                }
                if (TM) {
                    const T lx0 = wlx[l][1];
                    const T ly0 = d2(wez[l][0], wez[l][1], wez[l][2]);
                    const T lxy = d2(wlx[l][0], lx0, wlx[l][2]);
                    if (!DELTA) {
                        nv[2] = a_tm_b(c.czx, c.czy, c.czz, lx0, ly0, lxy, wc[l][0][2]);
                        nc[2] = wc[l][0][2];
                    } else {
                        nv[2] = a_tm(c.czx, c.czy, c.czz, lx0, ly0, lxy);
                        nc[2] = wc[l][0][2] + nv[2];
                    }
                }
                // Chebyshev form: nv holds b + A x; the residual r = nv - x
                // updates the increment d and the iterate x + d
                T rr[3] = {T(0), T(0), T(0)}, nd[3] = {T(0), T(0), T(0)};
                if (CHEB) {
                    const T xo[3] = {wex[l][1], wey[l][0], wez[l][1]};
#pragma unroll
                    for (int q = 0; q < 3; q++) {
                        if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
                        const int bk = q < 2 ? 0 : 1;
                        rr[q] = nv[q] - xo[q];
                        nd[q] = fmad(a.cheb[bk][0][l - 1], wd[l][0][q], a.cheb[bk][1][l - 1] * rr[q]);
                        nv[q] = xo[q] + nd[q];
                    }
                }
                if (l < K) {
#pragma unroll
                    for (int q = 0; q < 3; q++) {
                        if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
                        out[l][q] = nv[q];
                        wc[l][0][q] = nc[q];   // carried value of this row, read by level l+1 next step
                        if (CHEB) wd[l][0][q] = nd[q];
                    }
                    if (BOTH) *reinterpret_cast<Triple<T> *>(&xq[l][pw][i + 1]) = Triple<T>{nv[1], nv[2], nv[0]};
                    else if (TE) xp[l][pw][i + 1] = Pair<T>{nv[0], nv[1]};
                    else xz[l][pw][i + 1] = nv[2];
                } else if (outcol && r >= Y0 && r < rend) {
                    const unsigned o = (unsigned)(r * nx + gxi) * (unsigned)sizeof(T);
                    if (resid) {
                        if (TE) {
                            const double d0 = CHEB ? (double)rr[0] : DELTA ? (double)nv[0] : (double)nv[0] - (double)wex[l][1];
                            const double d1 = CHEB ? (double)rr[1] : DELTA ? (double)nv[1] : (double)nv[1] - (double)wey[l][0];
                            rte += d0 * d0 + d1 * d1;
                        }
                        if (TM) {
                            const double d2 = CHEB ? (double)rr[2] : DELTA ? (double)nv[2] : (double)nv[2] - (double)wez[l][1];
                            rtm += d2 * d2;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < 3; q++) {
                        if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
                        if (store) {
                            st_off(a.x_out[q], o, nv[q]);
                            if (DELTA) st_off(a.s_out[q], o, nc[q]);
                            if (CHEB) st_off(a.s_out[q], o, nd[q]);
                        }
                        if (last) st_off_nt(a.E[q], o, pe[ps][q] + (DELTA ? nc[q] : nv[q]));
                    }
                }
            }
        }
        // level 0: the row loaded for this step
        if (ALL || t < Y0 + L + K) {
#pragma unroll
            for (int q = 0; q < 3; q++) {
                if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
                out[0][q] = px[ps][q];
                wc[0][0][q] = pc[ps][q];
                if (CHEB) wd[0][0][q] = first ? T(0) : pd[ps][q];
            }
            if (BOTH) *reinterpret_cast<Triple<T> *>(&xq[0][pw][i + 1]) = Triple<T>{px[ps][1], px[ps][2], px[ps][0]};
            else if (TE) xp[0][pw][i + 1] = Pair<T>{px[ps][0], px[ps][1]};
            else xz[0][pw][i + 1] = px[ps][2];
            // shift; the tail receives row t+PF (in the unrolled body
            // unconditionally: a row past the end is a valid, unused row)
#pragma unroll
            for (int u = 0; u + 1 < PF; u++)
#pragma unroll
                for (int q = 0; q < 3; q++) { px[u][q] = px[u + 1][q]; pc[u][q] = pc[u + 1][q]; pd[u][q] = pd[u + 1][q]; }
            if (ALL || t + PF < Y0 + L + K) load_row(px[PF - 1], pc[PF - 1], pd[PF - 1]);
        }
        if (last) {
#pragma unroll
            for (int u = 0; u + 1 < PF; u++)
#pragma unroll
                for (int q = 0; q < 3; q++) pe[u][q] = pe[u + 1][q];
            load_e(t + PF - 2 * K, pe[PF - 1]);
        }
        lds_barrier();
    };
    // groups of 6 steps: a multiple of the window periods (2 and 3), of the
    // LDS double buffer and of the prefetch depth
    using A = std::true_type;
    for (int t = tstart; t < tend; t += 6) {
        step(t + 0, A{}, std::integral_constant<int, 0>{});
        step(t + 1, A{}, std::integral_constant<int, 1>{});
        step(t + 2, A{}, std::integral_constant<int, 2>{});
        step(t + 3, A{}, std::integral_constant<int, 3>{});
        step(t + 4, A{}, std::integral_constant<int, 4>{});
        step(t + 5, A{}, std::integral_constant<int, 5>{});
    }
    if (resid) {
        block_sum2<RX>(rte, rtm, sred);
        if (threadIdx.x == 0) {
            a.partial[2 * pidx] = rte;
            a.partial[2 * pidx + 1] = rtm;
        }
    }
    lds_barrier();   // the LDS rows are reused by the caller's next item
}

template <typename T, int BLK, int K, int FORM, int RX, int OM>
__global__ __launch_bounds__(RX) void k2_stream(Coef<T> c, SweepArgs<T> a, int flags, int L, int nsx, int nwg)
{
    if (a.skip && *a.skip) return;   // the block has met its stop test
    __shared__ __attribute__((aligned(16))) char lds[stream_lds_bytes<T, BLK, K, RX>()];
    __shared__ double sred[2 * RX / 64];
    stream_tile<T, BLK, K, FORM, RX, OM>(c, a, flags, L, nsx, xcd_map(blockIdx.x, nwg), blockIdx.x, lds, sred);
}

constexpr int SRX = 256;   // threads (columns) per workgroup strip

template <typename T, int BLK, int K, int FORM, int OM>
hipError_t stream_om(const Coef<T> &c, int flags, const SweepArgs<T> &a, hipStream_t s, int *nwg, int slots)
{
    constexpr int W = stream_width<SRX>(K);
    static std::atomic<int> resident[MX_MAX_DEVICES];
    if (slots <= 0)
        slots = per_device(resident, [] {
            int o = 0, dev = 0, cu = 0;
            (void)hipGetDevice(&dev);
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k2_stream<T, BLK, K, FORM, SRX, OM>, SRX, 0) != hipSuccess || o < 1) o = 1;
            if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu < 1) cu = 256;
            return o * cu;
        });
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
    hipLaunchKernelGGL((k2_stream<T, BLK, K, FORM, SRX, OM>), dim3(n), dim3(SRX), 0, s, c, a, flags, L, nsx, n);
    return hipGetLastError();
}

template <typename T, int BLK, int K, int FORM>
hipError_t stream_k(const Coef<T> &c, int flags, const SweepArgs<T> &a, hipStream_t s, int *nwg, int slots)
{
    const int out = flags & (SW_LAST | SW_STORE | SW_RESID);
    if (out == SW_LAST) return stream_om<T, BLK, K, FORM, OM_LAST>(c, flags, a, s, nwg, slots);
    if (out == SW_STORE) return stream_om<T, BLK, K, FORM, OM_STORE>(c, flags, a, s, nwg, slots);
    if (out == (SW_STORE | SW_RESID)) return stream_om<T, BLK, K, FORM, OM_RESID>(c, flags, a, s, nwg, slots);
    return hipErrorInvalidValue;
}

// deepest pass (sweeps per pass) of a block set's kernel: the per-level
// register windows must leave two waves per SIMD (TE carries 2 components,
// TM one, both together 3; the delta and Chebyshev forms carry one more
// value per component and level); TM is capped at 16, the levels of the
// per-sweep factor table
template <typename T, int BLK, int FORM>
constexpr int stream_kmax()
{
    constexpr bool F32 = sizeof(T) == 4;
    if (FORM == FM_CHEB) return F32 ? (BLK == 1 ? 10 : BLK == 2 ? 16 : 6) : (BLK == 1 ? 4 : BLK == 2 ? 8 : 2);
    if (FORM == FM_DELTA) return F32 ? (BLK == 1 ? 12 : BLK == 2 ? 16 : 8) : (BLK == 1 ? 6 : BLK == 2 ? 10 : 3);
    return F32 ? (BLK == 1 ? 14 : BLK == 2 ? 16 : 9) : (BLK == 1 ? 7 : BLK == 2 ? 12 : 4);
}

template <typename T, int BLK, int FORM, int K>
hipError_t stream_kdisp(const Coef<T> &c, int k, int flags, const SweepArgs<T> &a, hipStream_t s, int *nwg,
                        int slots)
{
    if constexpr (K == 0) {
        return hipErrorInvalidValue;
    } else {
        if (k == K) return stream_k<T, BLK, K, FORM>(c, flags, a, s, nwg, slots);
        return stream_kdisp<T, BLK, FORM, K - 1>(c, k, flags, a, s, nwg, slots);
    }
}

// one pass of k sweeps over the TE (BLK 1) or the TM (BLK 2) block, or both
// (3), in iterate form FORM
template <typename T, int FORM, int BLK>
hipError_t launch(const Coef<T> &c, int k, int flags, const SweepArgs<T> &a, hipStream_t s, int *nwg, int slots)
{
    return stream_kdisp<T, BLK, FORM, stream_kmax<T, BLK, FORM>()>(c, k, flags, a, s, nwg, slots);
}

}  // namespace stream2d
}  // namespace mx
