// 3D mass-matrix sweep pass, K sweeps per pass over HBM (Alg 1 with A from
// eqs matrixA_1st..matrixA_last; the Chebyshev form of the accelerated
// solve), marching in z.
//
// The 33-point A of each component splits into quantities of one z plane
// (differences and averages across x and y) combined along z: e.g. the x
// component is
//   (A x)_x = a_yy Dyy X + a_zz Dzz X + a_yz Dzz(Dyy X) + o_xy avg_z(Dx Dy Y)
//           + o_xz (avg_y(Dx Z)(k) - avg_y(Dx Z)(k - 1)),
// so a sweep level needs only one plane of its input in LDS.  When plane p
// of a level's input arrives, its in-plane quantities are folded at once
// into the three outputs they touch (planes p - 1, p and p + 1): output
// p - 1 is then complete, and only two partial sums per column are carried
// instead of windows of the quantities themselves.  Every output is summed
// in the same order, ((from p - 1) + (from p)) + (from p + 1), whatever the
// pass depth, so passes of any depth give bitwise identical iterates.
//
// A workgroup of TX x TYT threads owns a column tile of TX x TY (TY = R TYT;
// each thread carries R consecutive rows, which share their neighbours'
// LDS reads).  Level l (1..K) computes plane t - 2l at march step t from
// the planes of level l - 1 that arrived at earlier steps (one barrier per
// step), and hands its newest plane to level l + 1 through a
// double-buffered LDS plane.  The valid columns shrink by one per level on
// each side, so a tile writes (TX - 2(K - 1)) x (TY - 2(K - 1)) columns;
// the level-0 plane is loaded with a one-cell ring.  The carried value (dE'
// in the standard form, the running sum in the delta form, dE' and the
// increment in the Chebyshev form) travels with the planes.
#include <algorithm>
#include <atomic>

#include "mx_internal.h"
#include "stencil2d.h"

namespace mx {
namespace {

__device__ __forceinline__ int wrapm(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

template <typename T>
struct P3 {
    T x, y, z;
};

template <typename T>
__device__ __forceinline__ P3<T> p3add(const P3<T> &a, const P3<T> &b)
{
    return P3<T>{a.x + b.x, a.y + b.y, a.z + b.z};
}

// z-independent factors of the three plane contributions, formed in FP64 on
// the host from the coefficients of A and rounded once
template <typename T>
struct Zc {
    // x, from planes p - 1 and p + 1: a01 X + a02 Dyy X + o2/6 DxDy Y
    //    (and - o1 rxz from p - 1); from p: (a00 - 2 a02) Dyy X - 2 a01 X
    //    + 2 o2/3 DxDy Y + o1 rxz
    T a01, a02, o2s, o1, b00, m01, o2c;
    // y: the same with the roles of x and y exchanged
    T a10, a12, o0, b11, m10;
    // z, from p: a20 Dxx Z + a21 Dyy Z + a22 DxxDyy Z - o1 szx - o0 szy;
    //    from p + 1: o1 szx + o0 szy
    T a20, a21, a22;
};

// in-plane quantities of one column of one plane (see the header comment)
template <typename T>
struct Q {
    T X, Y, Z;          // own values
    T lyyx, pxy, rxz;   // Dyy X, Dx Dy Y, avg_y(Dx Z)   (x component)
    T lxxy, pyx, ryz;   // Dxx Y, Dy Dx X, avg_x(Dy Z)   (y component)
    T lxxz, lyyz, lxyz; // Dxx Z, Dyy Z, Dyy Dxx Z       (z component)
    T szx, szy;         // avg_y(Dx' X), avg_x(Dy' Y)    (backward differences)
};

// average with weights (1, 4, 1)/6: f0 + (fm + fp - 2 f0)/6
template <typename T>
__device__ __forceinline__ T avg6(T fm, T f0, T fp)
{
    return fmad(d2(fm, f0, fp), T(1.0 / 6.0), f0);
}

// v[dj + 1][di + 1]: the 3 x 3 neighbourhood of the column
template <typename T>
__device__ __forceinline__ Q<T> inplane(const P3<T> (&v)[3][3])
{
    auto X = [&](int di, int dj) { return v[dj + 1][di + 1].x; };
    auto Y = [&](int di, int dj) { return v[dj + 1][di + 1].y; };
    auto Z = [&](int di, int dj) { return v[dj + 1][di + 1].z; };
    Q<T> q;
    q.X = X(0, 0);
    q.Y = Y(0, 0);
    q.Z = Z(0, 0);
    q.lyyx = d2(X(0, -1), q.X, X(0, 1));
    q.pxy = (Y(1, 0) - Y(1, -1)) - (q.Y - Y(0, -1));
    q.rxz = avg6(Z(1, -1) - Z(0, -1), Z(1, 0) - q.Z, Z(1, 1) - Z(0, 1));
    q.lxxy = d2(Y(-1, 0), q.Y, Y(1, 0));
    q.pyx = (X(0, 1) - X(-1, 1)) - (q.X - X(-1, 0));
    q.ryz = avg6(Z(-1, 1) - Z(-1, 0), Z(0, 1) - q.Z, Z(1, 1) - Z(1, 0));
    const T lxm = d2(Z(-1, -1), Z(0, -1), Z(1, -1)), lxp = d2(Z(-1, 1), Z(0, 1), Z(1, 1));
    q.lxxz = d2(Z(-1, 0), q.Z, Z(1, 0));
    q.lyyz = d2(Z(0, -1), q.Z, Z(0, 1));
    q.lxyz = d2(lxm, q.lxxz, lxp);
    q.szx = avg6(X(0, -1) - X(-1, -1), q.X - X(-1, 0), X(0, 1) - X(-1, 1));
    q.szy = avg6(Y(-1, 0) - Y(-1, -1), q.Y - Y(0, -1), Y(1, 0) - Y(1, -1));
    return q;
}

// contributions of plane p to the outputs at p + 1 (f0), p (f1), p - 1 (f2)
template <typename T>
__device__ __forceinline__ void fold(const Zc<T> &z, const Q<T> &q, P3<T> &f0, P3<T> &f1, P3<T> &f2)
{
    const T sx = fmad(z.o2s, q.pxy, fmad(z.a02, q.lyyx, z.a01 * q.X));
    const T sy = fmad(z.o2s, q.pyx, fmad(z.a12, q.lxxy, z.a10 * q.Y));
    f2 = P3<T>{sx, sy, fmad(z.o1, q.szx, z.o0 * q.szy)};
    f0 = P3<T>{fmad(-z.o1, q.rxz, sx), fmad(-z.o0, q.ryz, sy), T(0)};
    f1.x = fmad(z.o1, q.rxz, fmad(z.o2c, q.pxy, fmad(z.m01, q.X, z.b00 * q.lyyx)));
    f1.y = fmad(z.o0, q.ryz, fmad(z.o2c, q.pyx, fmad(z.m10, q.Y, z.b11 * q.lxxy)));
    f1.z = fmad(-z.o0, q.szy, fmad(-z.o1, q.szx, fmad(z.a22, q.lxyz, fmad(z.a21, q.lyyz, z.a20 * q.lxxz))));
}

template <typename T>
__device__ __forceinline__ T comp(const P3<T> &p, int q) { return q == 0 ? p.x : (q == 1 ? p.y : p.z); }
template <typename T>
__device__ __forceinline__ void setc(P3<T> &p, int q, T v)
{
    if (q == 0) p.x = v;
    else if (q == 1) p.y = v;
    else p.z = v;
}

// FORM: FM_STD (x_l = b + A x_(l-1)), FM_DELTA (d_l = A d_(l-1), s_l = s_(l-1)
// + d_l) or FM_CHEB (r = b + A x - x, d_l = f_l d_(l-1) + g_l r, x_l = x + d_l).
template <typename T, int K, int FORM, int TX, int TYT, int R>
__global__ __launch_bounds__(TX *TYT) void k3_stream(Coef<T> c, Zc<T> z, SweepArgs<T> a, int flags, int Lz)
{
    constexpr bool DELTA = FORM == FM_DELTA, CHEB = FORM == FM_CHEB;
    constexpr int NTH = TX * TYT, TY = TYT * R, LX = TX + 2, LY = TY + 2;
    constexpr int RING = 2 * (LX + TY), RPER = (RING + NTH - 1) / NTH;
    if (a.skip && *a.skip) return;   // the solve has met its stop test
    __shared__ P3<T> pl[K][2][LY][LX];   // [level][parity][y][x]
    __shared__ double sred[NTH / 64];
    const int nx = c.nx, ny = c.ny, nz = c.nz;
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const int nwg = gridDim.x * gridDim.y * gridDim.z;
    const int lin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const int tl = xcd_map(lin, nwg);
    const int gxy = gridDim.x * gridDim.y;
    constexpr int OX = TX - 2 * (K - 1), OY = TY - 2 * (K - 1);   // output columns of a tile
    const int X0 = (tl % gridDim.x) * OX, Y0 = ((tl % gxy) / gridDim.x) * OY;
    const int Z0 = (tl / gxy) * Lz, Z1 = min(nz, Z0 + Lz);
    const size_t plane = (size_t)nx * ny;
    // own columns: x = ux, rows uy0 + r, LDS rows ly0 + r
    const int ux = X0 - (K - 1) + tx, ly0 = 1 + ty * R, uy0 = Y0 - (K - 1) + ty * R;
    size_t own[R];
    bool outc[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        own[r] = (size_t)wrapm(uy0 + r, ny) * nx + wrapm(ux, nx);
        const int iy = ty * R + r;
        outc[r] = tx >= K - 1 && tx < TX - (K - 1) && iy >= K - 1 && iy < TY - (K - 1) && ux < nx && uy0 + r < ny;
    }
    // ring cells of the level-0 plane this thread loads
    size_t roff[RPER];
    int rcx[RPER], rcy[RPER];
#pragma unroll
    for (int u = 0; u < RPER; u++) {
        const int rr = tid + u * NTH;
        int cx = -1, cy = -1;
        if (rr < RING) {
            if (rr < LX) { cx = rr; cy = 0; }
            else if (rr < 2 * LX) { cx = rr - LX; cy = LY - 1; }
            else if (rr < 2 * LX + TY) { cx = 0; cy = rr - 2 * LX + 1; }
            else { cx = LX - 1; cy = rr - 2 * LX - TY + 1; }
        }
        rcx[u] = cx;
        rcy[u] = cy;
        roff[u] = cx < 0 ? 0 : (size_t)wrapm(Y0 - K + cy, ny) * nx + wrapm(X0 - K + cx, nx);
    }
    const bool first = flags & SW_FIRST;
    const T *xin[3], *cin[3];
#pragma unroll
    for (int q = 0; q < 3; q++) {
        xin[q] = first ? a.rhs[q] : a.x_in[q];
        cin[q] = (DELTA && !first) ? a.s_in[q] : a.rhs[q];
    }
    // prefetched level-0 plane (own columns, ring cells), carried values
    P3<T> px[R], pc[R], pd[R], pr[RPER];
    auto fetch = [&](int k) {
        const size_t zo = (size_t)wrapm(k, nz) * plane;
#pragma unroll
        for (int r = 0; r < R; r++) {
            px[r] = P3<T>{xin[0][zo + own[r]], xin[1][zo + own[r]], xin[2][zo + own[r]]};
            pc[r] = P3<T>{cin[0][zo + own[r]], cin[1][zo + own[r]], cin[2][zo + own[r]]};
            if (CHEB) {
                if (first) pd[r] = P3<T>{T(0), T(0), T(0)};
                else pd[r] = P3<T>{a.s_in[0][zo + own[r]], a.s_in[1][zo + own[r]], a.s_in[2][zo + own[r]]};
            }
        }
#pragma unroll
        for (int u = 0; u < RPER; u++)
            if (rcx[u] >= 0) pr[u] = P3<T>{xin[0][zo + roff[u]], xin[1][zo + roff[u]], xin[2][zo + roff[u]]};
    };
    // per level l (1..K) and row: partial sums of the outputs at planes p
    // (sa) and p + 1 (sb) after plane p of level l - 1 arrived, and the own
    // value (xp), carried value (cp) and increment (dp) of plane p, used when
    // output p completes; per level l (0..K-1): carried value (oc) and
    // increment (od) of the level's newest plane, for level l + 1
    const P3<T> zero3{T(0), T(0), T(0)};
    P3<T> sa[K + 1][R], sb[K + 1][R], xp[K + 1][R], cp[K + 1][R], dp[K + 1][R], oc[K + 1][R], od[K + 1][R];
#pragma unroll
    for (int l = 0; l <= K; l++)
#pragma unroll
        for (int r = 0; r < R; r++) sa[l][r] = sb[l][r] = xp[l][r] = cp[l][r] = dp[l][r] = oc[l][r] = od[l][r] = zero3;
    T pe[R][3];   // E of the next output plane (last pass)
#pragma unroll
    for (int r = 0; r < R; r++) pe[r][0] = pe[r][1] = pe[r][2] = T(0);
    const bool last = flags & SW_LAST, store = flags & SW_STORE, resid = flags & SW_RESID;
    double acc = 0.0;
    const int tbeg = Z0 - K, tend = Z1 + 2 * K;
    fetch(tbeg);
    for (int t = tbeg; t < tend; t++) {
        const int pw = (t - tbeg) & 1, prd = pw ^ 1;
#pragma unroll
        for (int l = K; l >= 1; l--) {
            // arrival of plane p = t - 2l + 1 of level l - 1 (written at the
            // previous step); it completes output o = p - 1 of level l
            const int p = t - 2 * l + 1, o = p - 1;
            if (p >= Z0 - (K - l + 1) && p < Z1 + (K - l + 1)) {
                const bool out_ok = o >= Z0 - (K - l) && o < Z1 + (K - l);
                P3<T> nb[R + 2][3];
#pragma unroll
                for (int j = 0; j < R + 2; j++)
#pragma unroll
                    for (int i = 0; i < 3; i++) nb[j][i] = pl[l - 1][prd][ly0 - 1 + j][tx + i];
#pragma unroll
                for (int r = 0; r < R; r++) {
                    P3<T> win[3][3];
#pragma unroll
                    for (int j = 0; j < 3; j++)
#pragma unroll
                        for (int i = 0; i < 3; i++) win[j][i] = nb[r + j][i];
                    const Q<T> q = inplane<T>(win);
                    P3<T> f0, f1, f2;
                    fold<T>(z, q, f0, f1, f2);
                    if (out_ok) {
                        const P3<T> ax = p3add(sa[l][r], f2);   // (A x) at plane o
                        const P3<T> xo = xp[l][r], co = cp[l][r];
                        P3<T> nv, nc = co, nd = zero3, rres = zero3;
#pragma unroll
                        for (int qq = 0; qq < 3; qq++) {
                            const T aq = comp(ax, qq);
                            T v = DELTA ? aq : comp(co, qq) + aq;
                            if (DELTA) setc(nc, qq, comp(co, qq) + v);
                            if (CHEB) {
                                const T rq = v - comp(xo, qq);
                                const T d = fmad(a.cheb[0][0][l - 1], comp(dp[l][r], qq), a.cheb[0][1][l - 1] * rq);
                                setc(rres, qq, rq);
                                setc(nd, qq, d);
                                v = comp(xo, qq) + d;
                            }
                            setc(nv, qq, v);
                        }
                        if (l < K) {
                            oc[l][r] = nc;
                            od[l][r] = nd;
                            pl[l][pw][ly0 + r][tx + 1] = nv;
                        } else if (outc[r] && o >= Z0 && o < Z1) {
                            const size_t off = (size_t)o * plane + own[r];
#pragma unroll
                            for (int qq = 0; qq < 3; qq++) {
                                if (resid) {
                                    const double dd = CHEB    ? (double)comp(rres, qq)
                                                      : DELTA ? (double)comp(nv, qq)
                                                              : (double)comp(nv, qq) - (double)comp(xo, qq);
                                    acc += dd * dd;
                                }
                                if (store) {
                                    a.x_out[qq][off] = comp(nv, qq);
                                    if (DELTA) a.s_out[qq][off] = comp(nc, qq);
                                    if (CHEB) a.s_out[qq][off] = comp(nd, qq);
                                }
                                if (last) a.E[qq][off] = pe[r][qq] + (DELTA ? comp(nc, qq) : comp(nv, qq));
                            }
                        }
                    }
                    sa[l][r] = p3add(sb[l][r], f1);
                    sb[l][r] = f0;
                    xp[l][r] = P3<T>{q.X, q.Y, q.Z};
                    cp[l][r] = oc[l - 1][r];
                    if (CHEB) dp[l][r] = od[l - 1][r];
                }
            }
        }
        // level 0: plane t (own columns and ring)
        if (t < Z1 + K) {
#pragma unroll
            for (int r = 0; r < R; r++) {
                oc[0][r] = pc[r];
                od[0][r] = pd[r];
                pl[0][pw][ly0 + r][tx + 1] = px[r];
            }
#pragma unroll
            for (int u = 0; u < RPER; u++)
                if (rcx[u] >= 0) pl[0][pw][rcy[u]][rcx[u]] = pr[u];
            if (t + 1 < Z1 + K) fetch(t + 1);
        }
        // E of the output plane of the next step
        if (last) {
            const int on = t + 1 - 2 * K;
            if (on >= Z0 && on < Z1)
#pragma unroll
                for (int r = 0; r < R; r++)
                    if (outc[r])
#pragma unroll
                        for (int qq = 0; qq < 3; qq++) pe[r][qq] = a.E[qq][(size_t)on * plane + own[r]];
        }
        lds_barrier();
    }
    if (resid) {
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        const int lane = tid & 63, wv = tid >> 6;
        __syncthreads();
        if (lane == 0) sred[wv] = acc;
        __syncthreads();
        if (tid == 0) {
            double s_ = 0.0;
            for (int q = 0; q < NTH / 64; q++) s_ += sred[q];
            a.partial[2 * lin] = s_;
            a.partial[2 * lin + 1] = 0.0;
        }
    }
}

template <typename T>
Zc<T> zcoef(const Coef<T> &c)
{
    auto d = [](T v) { return (double)v; };
    Zc<T> z;
    z.a01 = c.a3[0][1];
    z.a02 = c.a3[0][2];
    z.o2s = (T)(d(c.o3[2]) / 6.0);
    z.o1 = c.o3[1];
    z.b00 = (T)(d(c.a3[0][0]) - 2.0 * d(c.a3[0][2]));
    z.m01 = (T)(-2.0 * d(c.a3[0][1]));
    z.o2c = (T)(d(c.o3[2]) * (4.0 / 6.0));
    z.a10 = c.a3[1][0];
    z.a12 = c.a3[1][2];
    z.o0 = c.o3[0];
    z.b11 = (T)(d(c.a3[1][1]) - 2.0 * d(c.a3[1][2]));
    z.m10 = (T)(-2.0 * d(c.a3[1][0]));
    z.a20 = c.a3[2][0];
    z.a21 = c.a3[2][1];
    z.a22 = c.a3[2][2];
    return z;
}

// Number of z chunks of a launch with ncol column tiles: every workgroup
// marches Lz + 3K plane steps (its chunk and the pipeline's fill and
// drain), and the workgroups run in rounds of `slots` (the co-resident
// limit), so the pass takes about ceil(ncol nzc / slots) (Lz + 3K) plane
// steps; the count minimising that is taken (chunks of at least 8K planes).
inline int z_chunks(int ncol, int nz, int K, int slots)
{
    const int maxc = std::max(1, nz / (8 * K));
    int best = 1;
    double bt = 1e300;
    for (int n = 1; n <= maxc; n++) {
        const int Lz = (nz + n - 1) / n, nc = (nz + Lz - 1) / Lz;
        const double rounds = slots > 0 ? (double)(((int64_t)ncol * nc + slots - 1) / slots) : (double)ncol * nc;
        const double t = rounds * (Lz + 3 * K);
        if (t < bt * (1.0 - 1e-9)) { bt = t; best = nc; }
    }
    return best;
}

template <typename T, int K, int FORM, int TX, int TYT, int R>
hipError_t launch_k(const Coef<T> &c, int flags, const SweepArgs<T> &a, hipStream_t s, int *nwg)
{
    constexpr int OX = TX - 2 * (K - 1), OY = TYT * R - 2 * (K - 1);
    // the partial-sum buffer holds a slot per 64 x 4 cells of each plane
    static_assert(OX * OY >= 256, "tile too small for the partial-sum buffer");
    const auto kern = k3_stream<T, K, FORM, TX, TYT, R>;
    static std::atomic<int> slot_cache[MX_MAX_DEVICES];
    const int slots = per_device(slot_cache, [&]() {
        int dev = 0, cu = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)kern, TX * TYT, 0) != hipSuccess) return 0;
        return per * cu;
    });
    const int gx = (c.nx + OX - 1) / OX, gy = (c.ny + OY - 1) / OY;
    const int nzc = z_chunks(gx * gy, c.nz, K, slots);
    const int Lz = (c.nz + nzc - 1) / nzc;
    dim3 g(gx, gy, nzc);
    *nwg = g.x * g.y * g.z;
    hipLaunchKernelGGL(kern, g, dim3(TX * TYT), 0, s, c, zcoef(c), a, flags, Lz);
    return hipGetLastError();
}

// FP32 passes of two and three sweeps: 64 x 16 columns, one per thread
// (1024 threads; a tile's input rows touch about 3 cache lines for 60 output
// columns instead of 2 for 28): 512^3, three sweeps per pass, 2.11 against
// 2.33 ms per delta-form pass and 2.56 against 3.07 per Chebyshev pass; 64 x
// 8 threads with two rows each measured as 32 x 16.  FP64 passes of two
// sweeps: 64 x 16 columns on 64 x 8 threads with two rows each (a 64 x 16
// FP64 tile of 1024 threads spills), 3.49 against 4.00 ms per delta-form
// pass at 512^3; the FP64 Chebyshev form spills there and keeps 32 x 16.
// Single sweeps: 32 x 16 (two rows per thread on a 32 x 8 thread block
// measured the same at three sweeps per pass, 32 x 32 columns slower).
template <typename T, int FORM>
hipError_t launch_form(const Coef<T> &c, int k, int flags, const SweepArgs<T> &a, hipStream_t s, int *nwg)
{
    constexpr bool F32 = sizeof(T) == 4;
    switch (k) {
    case 1: return launch_k<T, 1, FORM, 32, 16, 1>(c, flags, a, s, nwg);
    case 2:
        if constexpr (F32) return launch_k<T, 2, FORM, 64, 16, 1>(c, flags, a, s, nwg);
        else if constexpr (FORM != FM_CHEB) return launch_k<T, 2, FORM, 64, 8, 2>(c, flags, a, s, nwg);
        else return launch_k<T, 2, FORM, 32, 16, 1>(c, flags, a, s, nwg);
    case 3:
        if constexpr (F32) return launch_k<T, 3, FORM, 64, 16, 1>(c, flags, a, s, nwg);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int stream3d_kmax(bool f64) { return f64 ? 2 : 3; }

template <typename T>
hipError_t launch_stream3d(const Coef<T> &c, int k, int form, int flags, const SweepArgs<T> &a, hipStream_t s,
                           int *nwg)
{
    if (k < 1 || k > stream3d_kmax(sizeof(T) == 8)) return hipErrorInvalidValue;
    if (form == FM_CHEB) return launch_form<T, FM_CHEB>(c, k, flags, a, s, nwg);
    if (form == FM_DELTA) return launch_form<T, FM_DELTA>(c, k, flags, a, s, nwg);
    return launch_form<T, FM_STD>(c, k, flags, a, s, nwg);
}

template hipError_t launch_stream3d<float>(const Coef<float> &, int, int, int, const SweepArgs<float> &, hipStream_t,
                                           int *);
template hipError_t launch_stream3d<double>(const Coef<double> &, int, int, int, const SweepArgs<double> &,
                                            hipStream_t, int *);

}  // namespace mx
