#pragma once
// Front and first sweep pass of the 2D step in one row-streaming pass
// (arXiv 1907.13088, Sec. 2.2.2 and Alg 1): the Faraday update of B, the
// binomial filter of the current and the auxiliary increment dE' (as in
// k2f_impl.h), followed at once by the first K sweeps x_l = dE' + A x_(l-1)
// of Alg 1 starting from x_0 = dE' (as in k2s_impl.h, standard form).
//
// A workgroup owns a strip of RX columns (one per thread) and walks down a
// chunk of rows.  At step t the front stage receives row t of E and of the
// old B, forms B^{n+1/2} of row t-1 and emits dE' of row s = t-3 in
// registers; that row is level 0 of the sweep pipeline at once, so dE' is
// read by the sweeps without a round trip through memory.  Sweep level l
// computes row s-2l, as in the separate pass.  The front's LDS rows (E,
// B^{n+1/2}, raw current) and the levels' LDS rows are separate double
// buffers: one barrier per step serves both stages.
//
// The pass writes B^{n+1/2} and dE' (read by the later passes) and the
// K-th iterate of its own rows and columns.  Every value is formed by the
// same operations in the same order as the separate front and sweep
// kernels, so the results equal theirs bitwise.  E is only read: the pass
// cannot also be the last one (E += x in place would race with the halo
// reads of neighbouring work items).
#include <algorithm>
#include <type_traits>

#include "k2f_impl.h"
#include "k2s_impl.h"

namespace mx {
namespace fused2d {

using front2d::avg6;
using front2d::binom;
using stream2d::Quad;
using stream2d::Triple;

// columns left of the first output column: the front's left halo plus one
// per sweep level, or 16 for 128-byte aligned output runs of RX - 32 columns
template <int P, int K, bool AL>
constexpr int fs_halo() { return AL ? 16 : (P > 1 ? P : 1) + K; }
template <int P, int K, int RX, bool AL>
constexpr int fs_width() { return AL ? RX - 32 : RX - (P > 1 ? P : 1) - (P > 2 ? P : 2) - 2 * K; }

template <typename T, int P, int K, int RX>
constexpr size_t fs_lds_bytes()
{
    return front2d::front_lds_bytes<T, P, RX>() + sizeof(Quad<T>) * (size_t)K * 2 * (RX + 2);
}

template <typename T, int P, int K, int RX, bool HASJ, bool AL, int PF>
__device__ __forceinline__ void fs_tile(const Coef<T> &c, const FrontArgs<T> &fa, const T *Bin0, const T *Bin1,
                                        const T *Bin2, const SweepArgs<T> &sa, int L, int nsx, int wid, void *lds)
{
    constexpr int HLF = P > 1 ? P : 1;            // front: dE' valid on [HLF, RX - HRF)
    constexpr int HRF = P > 2 ? P : 2;
    constexpr int H = fs_halo<P, K, AL>();
    constexpr int W = fs_width<P, K, RX, AL>();
    static_assert(H >= HLF + K && RX - H - W >= HRF + K, "the halo must cover the front and every level");
    constexpr int PADL = P > 1 ? P : 1;
    constexpr int PR = RX + 2 * PADL;
    constexpr int D = P - 2;                      // the current is loaded D rows ahead of E
    constexpr int NP = P > 0 ? P : 1;
    constexpr int PAD = RX + 2;
    T(*sE)[2][PR] = reinterpret_cast<T(*)[2][PR]>(lds);
    T(*sB)[3][PR] = reinterpret_cast<T(*)[3][PR]>((T *)lds + 2 * 2 * PR);
    T(*sJ)[3][PR] = reinterpret_cast<T(*)[3][PR]>((T *)lds + 2 * 5 * PR);
    Quad<T>(*xq)[2][PAD] =
        reinterpret_cast<Quad<T>(*)[2][PAD]>((char *)lds + front2d::front_lds_bytes<T, P, RX>());

    const int sx = wid % nsx, sy = wid / nsx;
    const int nx = c.nx, ny = c.ny;
    const int i = threadIdx.x;
    const int li = i + PADL;
    const int X0 = sx * W, Y0 = sy * L;
    L = std::min(L, c.ny - Y0);
    const int gxi = X0 - H + i;
    const int gx = front2d::wrapi(gxi, nx);
    const bool outcol = i >= H && i < H + W && gxi < nx;
    const int rend = std::min(Y0 + L, ny);
    const T sixth = c.lumped ? T(0) : T(1.0 / 6.0);
    const T es = fa.env_src;

    // ---- front state (k2f_impl.h) ----
    // rows in flight: a FIFO of PF register sets, head = row t (in the
    // unrolled steady state the shifts are register renaming)
    T pE[PF][3], pB[PF][3], pJ[PF][3];
#pragma unroll
    for (int u = 0; u < PF; u++)
#pragma unroll
        for (int q = 0; q < 3; q++) pE[u][q] = pB[u][q] = pJ[u][q] = T(0);
    T e1[3] = {T(0), T(0), T(0)}, bo1[3] = {T(0), T(0), T(0)}, bp1[3] = {T(0), T(0), T(0)};
    T by_w[3] = {T(0), T(0), T(0)}, byl_w[3] = {T(0), T(0), T(0)}, axbx_w[3] = {T(0), T(0), T(0)};
    T bz_w[3] = {T(0), T(0), T(0)}, dxbz_w[2] = {T(0), T(0)};
    T fy[NP][3][2];
#pragma unroll
    for (int k = 0; k < NP; k++)
#pragma unroll
        for (int q = 0; q < 3; q++) fy[k][q][0] = fy[k][q][1] = T(0);

    // ---- sweep state (k2s_impl.h, standard form) ----
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

    // front rows: dE' rows [Y0 - K, Y0 + L + K) feed the sweep levels
    const int Y0f = Y0 - K;
    const int tb = std::min(Y0f - 1, Y0f - 2 * P + 2);   // front steps from here
    const int tend = Y0 + L + 2 * K + 3;                 // the last level's last row is out
    // Every step runs both stages in the steady form (no row-range tests) in
    // groups of 6 from the even step at or before tb: a value for a row
    // outside a stage's or level's range feeds only rows outside the next
    // one's range, and every store tests its row.  (Steps with range tests
    // took 2.5 times the instructions of a steady step.)
    const int tstart = tb - (tb & 1);
    const unsigned rowb = (unsigned)nx * (unsigned)sizeof(T);
    const unsigned allb = rowb * (unsigned)ny;
    const unsigned colb = (unsigned)gx * (unsigned)sizeof(T);
    unsigned loe = (unsigned)front2d::wrapi(tstart, ny) * rowb, loj = (unsigned)front2d::wrapi(tstart + D, ny) * rowb;
    auto load = [&](T(&e)[3], T(&bb)[3], T(&j)[3]) {
        const unsigned oe = loe + colb;
#pragma unroll
        for (int q = 0; q < 3; q++) e[q] = ld_off(fa.E[q], oe);
        bb[0] = ld_off(Bin0, oe);
        bb[1] = ld_off(Bin1, oe);
        bb[2] = ld_off(Bin2, oe);
        loe += rowb;
        if (loe >= allb) loe -= allb;
        if constexpr (HASJ) {
            const unsigned oj = loj + colb;
#pragma unroll
            for (int q = 0; q < 3; q++) j[q] = ld_off(fa.J0[q], oj);
            loj += rowb;
            if (loj >= allb) loj -= allb;
        }
    };
#pragma unroll
    for (int u = 0; u < PF; u++) load(pE[u], pB[u], pJ[u]);

    // FRONT: the front stage runs; SW: the sweep stage runs (0 none, 1 some
    // levels with row-range tests, 2 every level)
    auto step = [&](const int t, auto par_tag, auto front_tag, auto sw_tag) {
        constexpr bool FRONT = decltype(front_tag)::value;
        constexpr int SW = decltype(sw_tag)::value;
        constexpr int PARC = decltype(par_tag)::value;   // compile-time parity, or -1
        const int pw = PARC >= 0 ? PARC : (t & 1);
        const int pr = pw ^ 1;
        T dep[3] = {T(0), T(0), T(0)};   // dE' of row t - 3 (all columns)
        if constexpr (FRONT) {
            const T e0[3] = {pE[0][0], pE[0][1], pE[0][2]};
            const T bo0[3] = {pB[0][0], pB[0][1], pB[0][2]};
            const T jr[3] = {pJ[0][0], pJ[0][1], pJ[0][2]};
            // shift; the tail receives row t+PF (a row past the end is a
            // valid, unused row)
#pragma unroll
            for (int u = 0; u + 1 < PF; u++)
#pragma unroll
                for (int q = 0; q < 3; q++) { pE[u][q] = pE[u + 1][q]; pB[u][q] = pB[u + 1][q]; pJ[u][q] = pJ[u + 1][q]; }
            load(pE[PF - 1], pB[PF - 1], pJ[PF - 1]);
            T bp0[3];
            {
                const T ezr = sE[pr][1][li + 1];
                bp0[0] = bo1[0] - c.tdy * (e0[2] - e1[2]);
                bp0[1] = bo1[1] + c.tdx * (ezr - e1[2]);
                const T eyr = sE[pr][0][li + 1];
                bp0[2] = bo1[2] - (c.tdx * (eyr - e1[1]) - c.tdy * (e0[0] - e1[0]));
            }
            {
                const T bxl = sB[pr][0][li - 1], bxr = sB[pr][0][li + 1];
                axbx_w[0] = axbx_w[1]; axbx_w[1] = axbx_w[2]; axbx_w[2] = avg6(bxl, bp1[0], bxr, sixth);
                byl_w[0] = byl_w[1]; byl_w[1] = byl_w[2]; byl_w[2] = sB[pr][1][li - 1];
                by_w[0] = by_w[1]; by_w[1] = by_w[2]; by_w[2] = bp1[1];
                dxbz_w[0] = dxbz_w[1]; dxbz_w[1] = bp1[2] - sB[pr][2][li - 1];
                bz_w[0] = bz_w[1]; bz_w[1] = bz_w[2]; bz_w[2] = bp1[2];
            }
            T jf[3] = {T(0), T(0), T(0)};
            if constexpr (HASJ) {
#pragma unroll
                for (int q = 0; q < 3; q++) {
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
            dep[0] = c.tdy * (bz_w[1] - bz_w[0]) - es * jf[0];
            dep[1] = -c.tdx * dxbz_w[0] - es * jf[1];
            {
                const T ay = avg6(by_w[0], by_w[1], by_w[2], sixth);
                const T ayl = avg6(byl_w[0], byl_w[1], byl_w[2], sixth);
                dep[2] = c.tdx * (ay - ayl) - c.tdy * (axbx_w[1] - axbx_w[0]) - es * jf[2];
            }
            const int r = t - 3;
            if (outcol && r >= Y0 && r < rend) {
                const unsigned o = (unsigned)(r * nx + gxi) * (unsigned)sizeof(T);
#pragma unroll
                for (int q = 0; q < 3; q++) st_off(fa.dEp[q], o, dep[q]);
            }
            sE[pw][0][li] = e0[1];
            sE[pw][1][li] = e0[2];
            sB[pw][0][li] = bp0[0];
            sB[pw][1][li] = bp0[1];
            sB[pw][2][li] = bp0[2];
            if constexpr (HASJ) {
                sJ[pw][0][li] = jr[0];
                sJ[pw][1][li] = jr[1];
                sJ[pw][2][li] = jr[2];
            }
            const int rb = t - 1;
            if (outcol && rb >= Y0 && rb < rend) {
                const unsigned o = (unsigned)(rb * nx + gxi) * (unsigned)sizeof(T);
#pragma unroll
                for (int q = 0; q < 3; q++) st_off(fa.B[q], o, bp0[q]);
            }
#pragma unroll
            for (int q = 0; q < 3; q++) { e1[q] = e0[q]; bo1[q] = bo0[q]; bp1[q] = bp0[q]; }
        }
        if constexpr (SW > 0) {
            const int s = t - 3;
            constexpr bool ALL = SW == 2;
#pragma unroll
            for (int l = K; l >= 1; l--) {
                const int rho = s - 2 * l + 1;
                if (ALL || (rho >= Y0 - K + (l - 1) && rho < Y0 + L + K - (l - 1))) {
                    const Quad<T> qm = xq[l - 1][pr][i];
                    const stream2d::Pair<T> qp = *reinterpret_cast<const stream2d::Pair<T> *>(&xq[l - 1][pr][i + 2]);
                    const T exm = qm.ex, eym = qm.ey, ezm = qm.ez, eyp = qp.x, ezp = qp.y;
                    const T exn = out[l - 1][0], eyn = out[l - 1][1], ezn = out[l - 1][2];
                    wex[l][0] = wex[l][1]; wex[l][1] = wex[l][2]; wex[l][2] = exn;
                    wg[l][0] = wg[l][1]; wg[l][1] = wg[l][2]; wg[l][2] = eyp - eyn;
                    wley[l][0] = wley[l][1]; wley[l][1] = d2(eym, eyn, eyp);
                    wh[l][0] = wh[l][1]; wh[l][1] = exn - exm;
                    wey[l][0] = wey[l][1]; wey[l][1] = eyn;
                    wez[l][0] = wez[l][1]; wez[l][1] = wez[l][2]; wez[l][2] = ezn;
                    wlx[l][0] = wlx[l][1]; wlx[l][1] = wlx[l][2]; wlx[l][2] = d2(ezm, ezn, ezp);
#pragma unroll
                    for (int q = 0; q < 3; q++) { wc[l][0][q] = wc[l][1][q]; wc[l][1][q] = wc[l - 1][0][q]; }
                }
                const int r = s - 2 * l;
                if (ALL || (r >= Y0 - K + l && r < Y0 + L + K - l)) {
                    T nv[3];
                    {
                        const T lyy = d2(wex[l][0], wex[l][1], wex[l][2]);
                        const T dg = wg[l][1] - wg[l][0];
                        const T dh = wh[l][1] - wh[l][0];
                        nv[0] = a_te_x_b(c.cxx, c.cxy, lyy, dg, wc[l][0][0]);
                        nv[1] = a_te_y_b(c.cyy, c.cxy, wley[l][0], dh, wc[l][0][1]);
                        const T lx0 = wlx[l][1];
                        const T ly0 = d2(wez[l][0], wez[l][1], wez[l][2]);
                        const T lxy = d2(wlx[l][0], lx0, wlx[l][2]);
                        nv[2] = a_tm_b(c.czx, c.czy, c.czz, lx0, ly0, lxy, wc[l][0][2]);
                    }
                    if (l < K) {
#pragma unroll
                        for (int q = 0; q < 3; q++) out[l][q] = nv[q];
                        *reinterpret_cast<Triple<T> *>(&xq[l][pw][i + 1]) = Triple<T>{nv[1], nv[2], nv[0]};
                    } else if (outcol && r >= Y0 && r < rend) {
                        const unsigned o = (unsigned)(r * nx + gxi) * (unsigned)sizeof(T);
#pragma unroll
                        for (int q = 0; q < 3; q++) st_off(sa.x_out[q], o, nv[q]);
                    }
                }
            }
            // level 0: dE' of row s
            if (ALL || s < Y0 + L + K) {
#pragma unroll
                for (int q = 0; q < 3; q++) { out[0][q] = dep[q]; wc[0][0][q] = dep[q]; }
                *reinterpret_cast<Triple<T> *>(&xq[0][pw][i + 1]) = Triple<T>{dep[1], dep[2], dep[0]};
            }
        }
        lds_barrier();
    };
    using TT = std::true_type;
    using S2 = std::integral_constant<int, 2>;
    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    // groups of 6 steps: a multiple of the window periods 2 and 3, of the
    // LDS double buffers and of the prefetch parity
    for (int t = tstart; t < tend; t += 6) {
        step(t + 0, P0{}, TT{}, S2{});
        step(t + 1, P1{}, TT{}, S2{});
        step(t + 2, P0{}, TT{}, S2{});
        step(t + 3, P1{}, TT{}, S2{});
        step(t + 4, P0{}, TT{}, S2{});
        step(t + 5, P1{}, TT{}, S2{});
    }
    lds_barrier();
}

template <typename T, int P, int K, int RX, bool HASJ, bool AL, int PF, int WPE>
__global__ __launch_bounds__(RX, WPE) void k2_front_sweep(Coef<T> c, FrontArgs<T> fa, const T *Bin0, const T *Bin1,
                                                     const T *Bin2, SweepArgs<T> sa, int L, int nsx, int nwg)
{
    __shared__ __attribute__((aligned(16))) char lds[fs_lds_bytes<T, P, K, RX>()];
    fs_tile<T, P, K, RX, HASJ, AL, PF>(c, fa, Bin0, Bin1, Bin2, sa, L, nsx, xcd_map(blockIdx.x, nwg), lds);
}

template <typename T, int P, int K, int RX, bool HASJ, bool AL, int PF, int WPE>
hipError_t fs_launch(const Coef<T> &c, const FrontArgs<T> &fa, const T *const Bin[3], const SweepArgs<T> &sa,
                     hipStream_t s, int *nwg)
{
    constexpr int W = fs_width<P, K, RX, AL>();
    static std::atomic<int> resident[MX_MAX_DEVICES];
    const int slots = per_device(resident, [] {
        int o = 0, dev = 0, cu = 0;
        (void)hipGetDevice(&dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k2_front_sweep<T, P, K, RX, HASJ, AL, PF, WPE>, RX, 0) != hipSuccess || o < 1) o = 1;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu < 1) cu = 256;
        return o * cu;
    });
    const int nsx = (c.nx + W - 1) / W;
    int nsy = std::max(1, slots / nsx);
    nsy = std::min(nsy, c.ny);
    int L = (c.ny + nsy - 1) / nsy;
    L = std::max(L, std::min(c.ny, 4 * K));
    nsy = (c.ny + L - 1) / L;
    const int n = nsx * nsy;
    *nwg = n;
    hipLaunchKernelGGL((k2_front_sweep<T, P, K, RX, HASJ, AL, PF, WPE>), dim3(n), dim3(RX), 0, s, c, fa, Bin[0], Bin[1],
                       Bin[2], sa, L, nsx, n);
    return hipGetLastError();
}

// Launch shape: 256 columns per strip, 128-byte aligned output runs of 224
// columns (the pass is bound by HBM traffic more than the deep sweep passes
// are), two rows in flight per thread (4096^2, p = 3, K = 6: 281 against
// 287 us with one, 283 with three; 234 and 246 VGPRs, two waves per SIMD)
template <int K>
hipError_t fs_dispatch_k(const Coef<float> &c, int p, const FrontArgs<float> &fa, const float *const Bin[3],
                         const SweepArgs<float> &sa, hipStream_t s, int *nwg)
{
    if (fa.J0[0] == nullptr) return fs_launch<float, 0, K, 256, false, true, 2, 2>(c, fa, Bin, sa, s, nwg);
    switch (p) {
    case 0: return fs_launch<float, 0, K, 256, true, true, 2, 2>(c, fa, Bin, sa, s, nwg);
    case 1: return fs_launch<float, 1, K, 256, true, true, 2, 2>(c, fa, Bin, sa, s, nwg);
    case 2: return fs_launch<float, 2, K, 256, true, true, 2, 2>(c, fa, Bin, sa, s, nwg);
    case 3: return fs_launch<float, 3, K, 256, true, true, 2, 2>(c, fa, Bin, sa, s, nwg);
    case 4: return fs_launch<float, 4, K, 256, true, true, 2, 2>(c, fa, Bin, sa, s, nwg);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fused2d
}  // namespace mx
