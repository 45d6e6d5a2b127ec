// 3D kernels of the field step (arXiv 1907.13088, Sec. 2.2.1):
//   Faraday update ........ eqs faraday_x..z
//   current filter ........ p passes of (1,2,1)/4 along x, y and z
//   auxiliary increment ... eqs ampere_aux_x..z
//   mass-matrix sweep ..... Alg 1 with A from eqs matrixA_1st..matrixA_last
// One thread per cell, 64 x 4 threads per workgroup along x and y, one z
// plane per workgroup row of the grid; neighbour values come through the
// vector caches.
#include <algorithm>

#include "mx_internal.h"

namespace mx {
namespace {

constexpr int NT = 256;
constexpr int BXT = 64, BYT = 4;

__device__ __forceinline__ int wrap1(int i, int n)
{
    // i is within one period of [0, n)
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

struct Idx3 {
    int nx, ny, nz;
    int i, j, k;
    __device__ __forceinline__ size_t at(int di, int dj, int dk) const
    {
        const int x = wrap1(i + di, nx), y = wrap1(j + dj, ny), z = wrap1(k + dk, nz);
        return ((size_t)z * ny + y) * nx + x;
    }
};

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
        for (int q = 0; q < NT / 64; q++) { a += sh[2 * q]; b += sh[2 * q + 1]; }
    }
}

// Tile (x, y, z-chunk) of this workgroup: tiles are numbered x-fastest and
// dealt to the XCDs in contiguous ranges, so that a tile and its x and y
// neighbours mostly share one L2.
__device__ __forceinline__ int3 tile_of_block()
{
    const int n = gridDim.x * gridDim.y * gridDim.z;
    const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const int t = xcd_map(b, n);
    const int gxy = gridDim.x * gridDim.y;
    return make_int3(t % gridDim.x, (t % gxy) / gridDim.x, t / gxy);
}

__device__ __forceinline__ bool cell(int nx, int ny, Idx3 &id)
{
    const int tx = threadIdx.x & (BXT - 1), ty = threadIdx.x / BXT;
    const int3 tile = tile_of_block();
    id.i = tile.x * BXT + tx;
    id.j = tile.y * BYT + ty;
    id.k = tile.z;
    return id.i < nx && id.j < ny;
}

// alpha along an axis in "1 + small" form: f + (f- + f+ - 2 f)/6
template <typename T>
__device__ __forceinline__ T avg(T fm, T f0, T fp, int lumped)
{
    return lumped ? f0 : f0 + (fm + fp - T(2) * f0) * T(1.0 / 6.0);
}

template <typename T>
__global__ __launch_bounds__(NT) void k3_filter_axis(Coef<T> c, int axis, const T *src, T *dst)
{
    Idx3 id{c.nx, c.ny, c.nz, 0, 0, 0};
    if (!cell(c.nx, c.ny, id)) return;
    const int di = axis == 0, dj = axis == 1, dk = axis == 2;
    dst[id.at(0, 0, 0)] = T(0.25) * src[id.at(-di, -dj, -dk)] + T(0.5) * src[id.at(0, 0, 0)]
                        + T(0.25) * src[id.at(di, dj, dk)];
}

// B^{n+1/2} = B^{n-1/2} - dt curl E^n, in place (reads only E neighbours)
template <typename T>
__global__ __launch_bounds__(NT) void k3_faraday(Coef<T> c, const T *Ex, const T *Ey, const T *Ez,
                                                 T *Bx, T *By, T *Bz)
{
    Idx3 id{c.nx, c.ny, c.nz, 0, 0, 0};
    if (!cell(c.nx, c.ny, id)) return;
    const size_t o = id.at(0, 0, 0);
    const T ex = Ex[o], ey = Ey[o], ez = Ez[o];
    Bx[o] -= c.tdy * (Ez[id.at(0, 1, 0)] - ez) - c.tdz * (Ey[id.at(0, 0, 1)] - ey);
    By[o] -= c.tdz * (Ex[id.at(0, 0, 1)] - ex) - c.tdx * (Ez[id.at(1, 0, 0)] - ez);
    Bz[o] -= c.tdx * (Ey[id.at(1, 0, 0)] - ey) - c.tdy * (Ex[id.at(0, 1, 0)] - ex);
}

// dE' = dt curl(Lambda B^{n+1/2}) - 4 pi dt env Jf
template <typename T>
__global__ __launch_bounds__(NT) void k3_rhs(Coef<T> c, const T *Bx, const T *By, const T *Bz,
                                             const T *Jx, const T *Jy, const T *Jz, T env_src,
                                             T *dx_, T *dy_, T *dz_, double *partial)
{
    __shared__ double sred[2 * NT / 64];
    Idx3 id{c.nx, c.ny, c.nz, 0, 0, 0};
    const bool ok = cell(c.nx, c.ny, id);
    double acc = 0.0, dummy = 0.0;
    if (ok) {
        const int L = c.lumped;
        // alpha_z Bz at (i, j) and (i, j-1), (i-1, j)
        auto azBz = [&](int di, int dj) {
            return avg(Bz[id.at(di, dj, -1)], Bz[id.at(di, dj, 0)], Bz[id.at(di, dj, 1)], L);
        };
        // alpha_y By at (i, k), (i-1, k), (i, k-1)
        auto ayBy = [&](int di, int dk) {
            return avg(By[id.at(di, -1, dk)], By[id.at(di, 0, dk)], By[id.at(di, 1, dk)], L);
        };
        // alpha_x Bx at (j, k), (j-1, k), (j, k-1)
        auto axBx = [&](int dj, int dk) {
            return avg(Bx[id.at(-1, dj, dk)], Bx[id.at(0, dj, dk)], Bx[id.at(1, dj, dk)], L);
        };
        const T azbz = azBz(0, 0), ayby = ayBy(0, 0), axbx = axBx(0, 0);
        const T cx = c.tdy * (azbz - azBz(0, -1)) - c.tdz * (ayby - ayBy(0, -1));
        const T cy = c.tdz * (axbx - axBx(0, -1)) - c.tdx * (azbz - azBz(-1, 0));
        const T cz = c.tdx * (ayby - ayBy(-1, 0)) - c.tdy * (axbx - axBx(-1, 0));
        const size_t o = id.at(0, 0, 0);
        const T vx = cx - (Jx ? env_src * Jx[o] : T(0));
        const T vy = cy - (Jy ? env_src * Jy[o] : T(0));
        const T vz = cz - (Jz ? env_src * Jz[o] : T(0));
        dx_[o] = vx; dy_[o] = vy; dz_[o] = vz;
        acc = (double)vx * vx + (double)vy * vy + (double)vz * vz;
    }
    if (partial != nullptr) {
        block_sum2(acc, dummy, sred);
        if (threadIdx.x == 0) {
            const size_t wg = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            partial[2 * wg] = acc;
            partial[2 * wg + 1] = 0.0;
        }
    }
}

// (A x)_component at a cell, 33-point stencil per component (eqs
// matrixA_1st..matrixA_last).  X, Y, Z(di, dj, dk) return the iterate's
// components at the cell offset by (di, dj, dk).
template <typename T, typename FX, typename FY, typename FZ>
__device__ __forceinline__ void apply_A3(const Coef<T> &c, FX &&X, FY &&Y, FZ &&Z, T &ax, T &ay, T &az)
{
    const int L = 0;
    // second difference of F along axis e at offset d
    auto d2 = [&](auto &&F, int di, int dj, int dk, int ei, int ej, int ek) {
        return F(di + ei, dj + ej, dk + ek) + F(di - ei, dj - ej, dk - ek) - T(2) * F(di, dj, dk);
    };
    // --- x component: A_xx X + A_xy Y + A_xz Z
    {
        const T dyy = d2(X, 0, 0, 0, 0, 1, 0);
        const T dzz = d2(X, 0, 0, 0, 0, 0, 1);
        const T dyyzz = d2(X, 0, 1, 0, 0, 0, 1) + d2(X, 0, -1, 0, 0, 0, 1) - T(2) * dzz;
        // Dbar_x Dbar_y Y at (i+1/2, j, k+dk): Y at (i, j+1/2, k)
        auto dxdyY = [&](int dk) { return (Y(1, 0, dk) - Y(1, -1, dk)) - (Y(0, 0, dk) - Y(0, -1, dk)); };
        auto dxdzZ = [&](int dj) { return (Z(1, dj, 0) - Z(1, dj, -1)) - (Z(0, dj, 0) - Z(0, dj, -1)); };
        ax = c.a3[0][0] * dyy + c.a3[0][1] * dzz + c.a3[0][2] * dyyzz
           + c.o3[2] * avg(dxdyY(-1), dxdyY(0), dxdyY(1), L)
           + c.o3[1] * avg(dxdzZ(-1), dxdzZ(0), dxdzZ(1), L);
    }
    // --- y component: A_yy Y + A_yx X + A_yz Z
    {
        const T dzz = d2(Y, 0, 0, 0, 0, 0, 1);
        const T dxx = d2(Y, 0, 0, 0, 1, 0, 0);
        const T dzzxx = d2(Y, 1, 0, 0, 0, 0, 1) + d2(Y, -1, 0, 0, 0, 0, 1) - T(2) * dzz;
        auto dydxX = [&](int dk) { return (X(0, 1, dk) - X(-1, 1, dk)) - (X(0, 0, dk) - X(-1, 0, dk)); };
        auto dydzZ = [&](int di) { return (Z(di, 1, 0) - Z(di, 1, -1)) - (Z(di, 0, 0) - Z(di, 0, -1)); };
        ay = c.a3[1][0] * dzz + c.a3[1][1] * dxx + c.a3[1][2] * dzzxx
           + c.o3[2] * avg(dydxX(-1), dydxX(0), dydxX(1), L)
           + c.o3[0] * avg(dydzZ(-1), dydzZ(0), dydzZ(1), L);
    }
    // --- z component: A_zz Z + A_zx X + A_zy Y
    {
        const T dxx = d2(Z, 0, 0, 0, 1, 0, 0);
        const T dyy = d2(Z, 0, 0, 0, 0, 1, 0);
        const T dxxyy = d2(Z, 0, 1, 0, 1, 0, 0) + d2(Z, 0, -1, 0, 1, 0, 0) - T(2) * dxx;
        auto dzdxX = [&](int dj) { return (X(0, dj, 1) - X(-1, dj, 1)) - (X(0, dj, 0) - X(-1, dj, 0)); };
        auto dzdyY = [&](int di) { return (Y(di, 0, 1) - Y(di, -1, 1)) - (Y(di, 0, 0) - Y(di, -1, 0)); };
        az = c.a3[2][0] * dxx + c.a3[2][1] * dyy + c.a3[2][2] * dxxyy
           + c.o3[1] * avg(dzdxX(-1), dzdxX(0), dzdxX(1), L)
           + c.o3[0] * avg(dzdyY(-1), dzdyY(0), dzdyY(1), L);
    }
}

// One sweep pass, marching in z.  A workgroup of ZX x ZY threads owns a
// ZX x ZY column tile and walks down a chunk of z planes; the iterate's
// planes k-1, k, k+1 of the tile plus a one-cell halo in x and y sit in LDS
// (three rotating plane slots), so each cell of the iterate is read from
// HBM once per pass plus the halo.  Plane k+2 is prefetched into registers
// while plane k is computed.
constexpr int ZX = 64, ZY = 8, ZT = ZX * ZY;
constexpr int PX = ZX + 2, PY = ZY + 2, PCELLS = PX * PY;
constexpr int PLOAD = (PCELLS + ZT - 1) / ZT;   // halo-tile cells per thread

// FORM: FM_STD (Alg 1), FM_DELTA, or FM_CHEB (the Chebyshev sweep: with
// b + A x formed as in Alg 1, r = (b + A x) - x, d = f d_prev + g r and
// x + d; the increment of the own cell passes in and out through s_in and
// s_out, and f, g of this sweep are cheb[0][0][0], cheb[0][1][0]).
template <typename T, int FORM>
__global__ __launch_bounds__(ZT) void k3_sweep(Coef<T> c, SweepArgs<T> a, int flags, int Lz)
{
    constexpr bool DELTA = FORM == FM_DELTA, CHEB = FORM == FM_CHEB;
    if (a.skip && *a.skip) return;   // the solve has met its stop test
    __shared__ T pl[3][3][PY][PX];   // [slot][component][y][x]
    __shared__ double sred[2 * ZT / 64];
    const int nx = c.nx, ny = c.ny, nz = c.nz;
    const int tid = threadIdx.x, tx = tid % ZX, ty = tid / ZX;
    const int3 tile = tile_of_block();
    const int X0 = tile.x * ZX, Y0 = tile.y * ZY;
    const int Z0 = tile.z * Lz, Z1 = min(nz, Z0 + Lz);
    const int gx = X0 + tx, gy = Y0 + ty;
    const bool out = gx < nx && gy < ny;
    const bool first = flags & SW_FIRST;
    const T *xin[3], *cin[3];
    for (int q = 0; q < 3; q++) {
        xin[q] = first ? a.rhs[q] : a.x_in[q];
        cin[q] = (DELTA && !first) ? a.s_in[q] : a.rhs[q];   // carried: dE' (standard), running sum (delta)
    }
    const size_t plane = (size_t)nx * ny;
    // halo-tile cell offsets within a plane, fixed for the whole walk
    size_t hoff[PLOAD];
    int hidx[PLOAD];
    for (int u = 0; u < PLOAD; u++) {
        const int idx = tid + u * ZT;
        hidx[u] = idx < PCELLS ? idx : -1;
        const int ix = idx % PX, iy = idx / PX;
        // full modulo: a tile may be wider than the grid
        const int hx = ((X0 - 1 + ix) % nx + nx) % nx, hy = ((Y0 - 1 + iy) % ny + ny) % ny;
        hoff[u] = (size_t)hy * nx + hx;
    }
    T pre[PLOAD][3];
    auto fetch = [&](int k) {
        const size_t zo = (size_t)wrap1(k, nz) * plane;
        for (int u = 0; u < PLOAD; u++)
            if (hidx[u] >= 0)
                for (int q = 0; q < 3; q++) pre[u][q] = xin[q][zo + hoff[u]];
    };
    auto deposit = [&](int slot) {
        for (int u = 0; u < PLOAD; u++)
            if (hidx[u] >= 0)
                for (int q = 0; q < 3; q++) (&pl[slot][q][0][0])[hidx[u]] = pre[u][q];
    };
    const size_t own = (size_t)(out ? gy : 0) * nx + (out ? gx : 0);
    T cnext[3] = {T(0), T(0), T(0)}, dnext[3] = {T(0), T(0), T(0)};
    auto fetch_own = [&](int k) {
        if (!out || k >= Z1) return;
        for (int q = 0; q < 3; q++) {
            cnext[q] = cin[q][(size_t)k * plane + own];
            // no increment before the first sweep (its factor is 0)
            if (CHEB) dnext[q] = first ? T(0) : a.s_in[q][(size_t)k * plane + own];
        }
    };

    int sm = 0, s0 = 1, sp = 2;   // slots of planes k-1, k, k+1
    fetch(Z0 - 1);
    deposit(sm);
    fetch(Z0);
    deposit(s0);
    fetch(Z0 + 1);
    fetch_own(Z0);
    double acc = 0.0, dummy = 0.0;
    for (int k = Z0; k < Z1; k++) {
        deposit(sp);
        const T cown[3] = {cnext[0], cnext[1], cnext[2]};
        const T down[3] = {dnext[0], dnext[1], dnext[2]};
        __syncthreads();
        if (k + 2 <= Z1) fetch(k + 2);
        fetch_own(k + 1);
        if (out) {
            auto at = [&](int q) {
                return [&, q](int di, int dj, int dk) {
                    const int slot = dk < 0 ? sm : (dk > 0 ? sp : s0);
                    return pl[slot][q][ty + 1 + dj][tx + 1 + di];
                };
            };
            T ax, ay, az;
            apply_A3(c, at(0), at(1), at(2), ax, ay, az);
            const size_t o = (size_t)k * plane + own;
            T v[3] = {DELTA ? ax : cown[0] + ax, DELTA ? ay : cown[1] + ay, DELTA ? az : cown[2] + az};
            T nd[3] = {T(0), T(0), T(0)}, rr[3] = {T(0), T(0), T(0)};
            if (CHEB) {
                const T f = a.cheb[0][0][0], gr = a.cheb[0][1][0];
                for (int q = 0; q < 3; q++) {
                    const T xo = pl[s0][q][ty + 1][tx + 1];
                    rr[q] = v[q] - xo;
                    nd[q] = fma(f, down[q], gr * rr[q]);
                    v[q] = xo + nd[q];
                }
            }
            for (int q = 0; q < 3; q++) {
                if (flags & SW_RESID) {
                    const double d = CHEB ? (double)rr[q]
                                   : DELTA ? (double)v[q] : (double)v[q] - (double)pl[s0][q][ty + 1][tx + 1];
                    acc += d * d;
                }
                const T sum = DELTA ? cown[q] + v[q] : T(0);
                if (flags & SW_STORE) {
                    a.x_out[q][o] = v[q];
                    if (DELTA) a.s_out[q][o] = sum;
                    if (CHEB) a.s_out[q][o] = nd[q];
                }
                if (flags & SW_LAST) a.E[q][o] += DELTA ? sum : v[q];
            }
        }
        __syncthreads();   // plane k-1 is read by everyone before its slot is refilled
        const int t = sm; sm = s0; s0 = sp; sp = t;
    }
    if (flags & SW_RESID) {
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        const int lane = tid & 63, w = tid >> 6;
        if (lane == 0) sred[w] = acc;
        __syncthreads();
        if (tid == 0) {
            double s_ = 0.0;
            for (int q = 0; q < ZT / 64; q++) s_ += sred[q];
            const size_t wg = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            a.partial[2 * wg] = s_;
            a.partial[2 * wg + 1] = 0.0;
        }
        (void)dummy;
    }
}

// Two sweeps per pass (FP32), marching in z.  A workgroup of YX x YY
// threads owns a YX x YY column tile; each thread carries its own column
// through both sweep levels: level 0 (the input iterate) is loaded by every
// thread, level 1 is computed by the threads one cell inside the tile edge,
// level 2 (the pass output) by those two cells inside, so the output tile is
// (YX - 4) x (YY - 4).  Level 1 lags level 0 by one plane and level 2 lags
// level 1 by one plane; each level keeps three plane slots in LDS.  The
// carried value (dE' in the standard form, the running sum in the delta
// form) of a thread's own cell passes from level 1 to level 2 in registers.
constexpr int YX = 64, YY = 16, YT = YX * YY;
constexpr int YOX = YX - 4, YOY = YY - 4;

template <typename T, bool DELTA>
__global__ __launch_bounds__(YT) void k3_sweep2(Coef<T> c, SweepArgs<T> a, int flags, int Lz)
{
    if (a.skip && *a.skip) return;   // the solve has met its stop test
    __shared__ T l0[3][3][YY][YX];   // [slot][component][y][x]
    __shared__ T l1[3][3][YY][YX];
    __shared__ double sred[YT / 64];
    const int nx = c.nx, ny = c.ny, nz = c.nz;
    const int tid = threadIdx.x, tx = tid % YX, ty = tid / YX;
    const int3 tile = tile_of_block();
    const int X0 = tile.x * YOX, Y0 = tile.y * YOY;
    const int Z0 = tile.z * Lz, Z1 = min(nz, Z0 + Lz);
    // own column (level 0 is loaded at every tile cell, wrapped)
    const int ux = X0 - 2 + tx, uy = Y0 - 2 + ty;
    const int gx = ((ux % nx) + nx) % nx, gy = ((uy % ny) + ny) % ny;
    const bool in1 = tx >= 1 && tx < YX - 1 && ty >= 1 && ty < YY - 1;
    const bool in2 = tx >= 2 && tx < YX - 2 && ty >= 2 && ty < YY - 2 && ux < nx && uy < ny;
    const bool first = flags & SW_FIRST;
    const T *xin[3], *cin[3];
    for (int q = 0; q < 3; q++) {
        xin[q] = first ? a.rhs[q] : a.x_in[q];
        cin[q] = (DELTA && !first) ? a.s_in[q] : a.rhs[q];
    }
    const size_t plane = (size_t)nx * ny;
    const size_t own = (size_t)gy * nx + gx;
    auto zoff = [&](int k) { return (size_t)((k % nz + nz) % nz) * plane; };
    auto slot = [](int k) { return ((k % 3) + 3) % 3; };

    T pre[3];
    auto fetch0 = [&](int k) {
        const size_t o = zoff(k) + own;
        for (int q = 0; q < 3; q++) pre[q] = xin[q][o];
    };
    // carried value of level 1 (plane k - 1) and of level 2 (plane k - 2)
    T c1[3] = {T(0), T(0), T(0)}, c2[3] = {T(0), T(0), T(0)}, x1own[3] = {T(0), T(0), T(0)};
    double acc = 0.0;
    const int kb = Z0 - 2, ke = Z1 + 1;   // level-0 planes of the walk
    fetch0(kb);
    for (int k = kb; k <= ke; k++) {
        {
            const int s0 = slot(k);
            for (int q = 0; q < 3; q++) l0[s0][q][ty][tx] = pre[q];
        }
        if (k + 1 <= ke) fetch0(k + 1);
        // the carried input of level 1 for plane k - 1 (own cell)
        T cin1[3] = {T(0), T(0), T(0)};
        const int k1 = k - 1, k2 = k - 2;
        const bool act1 = k1 >= Z0 - 1 && k1 <= Z1 && in1;
        if (act1) {
            const size_t o = zoff(k1) + own;
            for (int q = 0; q < 3; q++) cin1[q] = cin[q][o];
        }
        __syncthreads();
        // level 1, plane k - 1
        T n1[3] = {T(0), T(0), T(0)}, s1[3] = {T(0), T(0), T(0)};
        if (act1) {
            const int sm = slot(k1 - 1), s0 = slot(k1), sp = slot(k1 + 1);
            auto at = [&](int q) {
                return [&, q](int di, int dj, int dk) {
                    return l0[dk < 0 ? sm : (dk > 0 ? sp : s0)][q][ty + dj][tx + di];
                };
            };
            T ax, ay, az;
            apply_A3(c, at(0), at(1), at(2), ax, ay, az);
            const T av[3] = {ax, ay, az};
            for (int q = 0; q < 3; q++) {
                n1[q] = DELTA ? av[q] : cin1[q] + av[q];
                s1[q] = DELTA ? cin1[q] + n1[q] : cin1[q];
                l1[s0][q][ty][tx] = n1[q];
            }
        }
        __syncthreads();
        // level 2, plane k - 2 (inputs: level-1 planes k - 3 .. k - 1)
        if (k2 >= Z0 && k2 < Z1 && in2) {
            const int sm = slot(k2 - 1), s0 = slot(k2), sp = slot(k2 + 1);
            auto at = [&](int q) {
                return [&, q](int di, int dj, int dk) {
                    return l1[dk < 0 ? sm : (dk > 0 ? sp : s0)][q][ty + dj][tx + di];
                };
            };
            T ax, ay, az;
            apply_A3(c, at(0), at(1), at(2), ax, ay, az);
            const T av[3] = {ax, ay, az};
            const size_t o = (size_t)k2 * plane + (size_t)uy * nx + ux;
            for (int q = 0; q < 3; q++) {
                const T v = DELTA ? av[q] : c2[q] + av[q];
                const T sum = DELTA ? c2[q] + v : T(0);
                if (flags & SW_RESID) {
                    const double d = DELTA ? (double)v : (double)v - (double)x1own[q];
                    acc += d * d;
                }
                if (flags & SW_STORE) {
                    a.x_out[q][o] = v;
                    if (DELTA) a.s_out[q][o] = sum;
                }
                if (flags & SW_LAST) a.E[q][o] += DELTA ? sum : v;
            }
        }
        // level 1's own results of plane k - 1 become level 2's inputs next step
        for (int q = 0; q < 3; q++) { c2[q] = s1[q]; x1own[q] = n1[q]; }
    }
    if (flags & SW_RESID) {
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        const int lane = tid & 63, w = tid >> 6;
        if (lane == 0) sred[w] = acc;
        __syncthreads();
        if (tid == 0) {
            double s_ = 0.0;
            for (int q = 0; q < YT / 64; q++) s_ += sred[q];
            const size_t wg = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            a.partial[2 * wg] = s_;
            a.partial[2 * wg + 1] = 0.0;
        }
    }
}

dim3 grid3(int nx, int ny, int nz) { return dim3((nx + BXT - 1) / BXT, (ny + BYT - 1) / BYT, nz); }

}  // namespace

template <typename T>
hipError_t launch_filter3d(const Coef<T> &c, int passes, const T *const J0[3], T *const Jf[3],
                           T *const tmp[3], hipStream_t s)
{
    // 3 * passes axis sweeps per component, ping-ponging so the last lands in Jf
    const int total = 3 * passes;
    for (int q = 0; q < 3; q++) {
        if (total == 0) {
            hipMemcpyAsync(Jf[q], J0[q], sizeof(T) * (size_t)c.nx * c.ny * c.nz, hipMemcpyDeviceToDevice, s);
            continue;
        }
        const T *src = J0[q];
        for (int t = 0; t < total; t++) {
            T *dst = ((total - 1 - t) % 2 == 0) ? Jf[q] : tmp[q];
            hipLaunchKernelGGL((k3_filter_axis<T>), grid3(c.nx, c.ny, c.nz), dim3(NT), 0, s, c, t % 3, src, dst);
            src = dst;
        }
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_faraday3d(const Coef<T> &c, const T *const E[3], T *const B[3], hipStream_t s)
{
    hipLaunchKernelGGL((k3_faraday<T>), grid3(c.nx, c.ny, c.nz), dim3(NT), 0, s, c, E[0], E[1], E[2],
                       B[0], B[1], B[2]);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rhs3d(const Coef<T> &c, const T *const B[3], const T *const Jf[3], T env_src,
                        T *const dEp[3], double *partial, hipStream_t s, int *nwg)
{
    dim3 g = grid3(c.nx, c.ny, c.nz);
    *nwg = g.x * g.y * g.z;
    hipLaunchKernelGGL((k3_rhs<T>), g, dim3(NT), 0, s, c, B[0], B[1], B[2], Jf ? Jf[0] : nullptr,
                       Jf ? Jf[1] : nullptr, Jf ? Jf[2] : nullptr, env_src, dEp[0], dEp[1], dEp[2], partial);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep3d(const Coef<T> &c, int k, int form, int flags, const SweepArgs<T> &a,
                          hipStream_t s, int *nwg)
{
    const bool delta = form == FM_DELTA;
    if (form == FM_CHEB && k != 1) return hipErrorInvalidValue;   // the Chebyshev form runs one sweep per pass
    if constexpr (sizeof(T) == 4) {
        if (k == 2) {
        // enough workgroups for whole rounds of one per CU, chunks of >= 16 planes
        const int gx = (c.nx + YOX - 1) / YOX, gy = (c.ny + YOY - 1) / YOY;
        int nzc = std::max(1, std::min(c.nz / 16, (2 * 256 + gx * gy - 1) / (gx * gy)));
        const int Lz = (c.nz + nzc - 1) / nzc;
        nzc = (c.nz + Lz - 1) / Lz;
        dim3 g(gx, gy, nzc);
        *nwg = g.x * g.y * g.z;
        if (delta) hipLaunchKernelGGL((k3_sweep2<T, true>), g, dim3(YT), 0, s, c, a, flags, Lz);
        else hipLaunchKernelGGL((k3_sweep2<T, false>), g, dim3(YT), 0, s, c, a, flags, Lz);
        return hipGetLastError();
        }
    }
    if (k != 1) return hipErrorInvalidValue;
    // z chunks: enough workgroups for two per CU, each chunk at least 16 planes
    const int gx = (c.nx + ZX - 1) / ZX, gy = (c.ny + ZY - 1) / ZY;
    int nzc = std::max(1, std::min(c.nz / 16, (512 + gx * gy - 1) / (gx * gy)));
    const int Lz = (c.nz + nzc - 1) / nzc;
    nzc = (c.nz + Lz - 1) / Lz;
    dim3 g(gx, gy, nzc);
    *nwg = g.x * g.y * g.z;
    if (form == FM_CHEB) hipLaunchKernelGGL((k3_sweep<T, FM_CHEB>), g, dim3(ZT), 0, s, c, a, flags, Lz);
    else if (delta) hipLaunchKernelGGL((k3_sweep<T, FM_DELTA>), g, dim3(ZT), 0, s, c, a, flags, Lz);
    else hipLaunchKernelGGL((k3_sweep<T, FM_STD>), g, dim3(ZT), 0, s, c, a, flags, Lz);
    return hipGetLastError();
}

#define INST(T)                                                                                       \
    template hipError_t launch_filter3d<T>(const Coef<T> &, int, const T *const[3], T *const[3],      \
                                           T *const[3], hipStream_t);                                 \
    template hipError_t launch_faraday3d<T>(const Coef<T> &, const T *const[3], T *const[3], hipStream_t); \
    template hipError_t launch_rhs3d<T>(const Coef<T> &, const T *const[3], const T *const[3], T,     \
                                        T *const[3], double *, hipStream_t, int *);                   \
    template hipError_t launch_sweep3d<T>(const Coef<T> &, int, int, int, const SweepArgs<T> &, hipStream_t, int *);
INST(float)
INST(double)
#undef INST

}  // namespace mx
