// Particle coupling of the 2D field step (arXiv 1907.13088: the solver runs
// inside a particle-in-cell code whose force interpolation, deposition and
// push it leaves unchanged, Sec. 2; Gauss's law for E holds when the
// deposition conserves charge, Sec. 2 and Appendix A):
//   push ........ relativistic Boris scheme (Boris 1970) in E^n and
//                 B^n = B^{n-1/2} - (dt/2) curl E^n, c = 1
//   shapes ...... first-order B-spline at each component's staggered
//                 position (the lowest order of the paper's Table 1)
//   deposition .. Esirkepov's charge-conserving decomposition (Esirkepov
//                 2001), 2D with an out-of-plane current, added with
//                 floating-point atomics: in LDS when the windows of a
//                 workgroup's particles fit one tile (particles kept in cell
//                 order), then once per node into J; else directly into J
// One thread per particle.  Positions are at time level n, momenta
// u = gamma v at n - 1/2; after the call positions are at n + 1 (wrapped
// into [0, L)), momenta at n + 1/2, and J holds J^{n+1/2}.
//
// A particle moves less than one cell per axis per step: |v| < c and the
// time step obeys the CFL bound dt <= (1/dx^2 + 1/dy^2)^(-1/2) < min(dx, dy),
// so the 4 x 4 node window starting one node before the start cell covers
// both shapes.
#include "mx_internal.h"

namespace mx {
namespace {

constexpr int PT = 256;

template <typename T>
__device__ __forceinline__ T shape1(T d)
{
    d = fabs(d);
    return d < T(1) ? T(1) - d : T(0);
}

__device__ __forceinline__ int wrapn(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

// the same for indices within a few cells of [0, n): no division
__device__ __forceinline__ int wrapc(int i, int n)
{
    if (i >= 0 && i < n) return i;
    const int j = i < 0 ? i + n : i - n;
    return (j >= 0 && j < n) ? j : wrapn(i, n);
}

// LDS accumulation tile of the deposition (nodes); rows and components
// padded so that neighbouring nodes of different rows or components fall in
// different LDS banks
constexpr int TWX = 32, TWY = 32, TPX = TWX + 1, TPC = TWY * TPX + 3;
// window contributions of one particle: J_x on 3 x 4 nodes, J_y on 4 x 3,
// J_z on 4 x 4
constexpr int NCON = 40;

// min and max of v over the workgroup (valid in every thread)
__device__ __forceinline__ void block_minmax(int &vmin, int &vmax, int *sh)
{
    for (int off = 32; off > 0; off >>= 1) {
        vmin = min(vmin, __shfl_xor(vmin, off, 64));
        vmax = max(vmax, __shfl_xor(vmax, off, 64));
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) { sh[2 * w] = vmin; sh[2 * w + 1] = vmax; }
    __syncthreads();
    vmin = sh[0];
    vmax = sh[1];
    for (int q = 1; q < PT / 64; q++) { vmin = min(vmin, sh[2 * q]); vmax = max(vmax, sh[2 * q + 1]); }
}

template <typename T>
__global__ __launch_bounds__(PT) void k_pic_push(PicArgs<T> a)
{
    __shared__ T tile[3 * TPC];
    __shared__ int sh[2 * PT / 64];
    const int64_t p = (int64_t)blockIdx.x * PT + threadIdx.x;
    const bool live = p < a.np;
    const int nx = a.nx, ny = a.ny;
    const T dx = a.dx, dy = a.dy, dt = a.dt, th = a.th;
    const T x0 = live ? a.x[p] : T(0), y0 = live ? a.y[p] : T(0);
    const T *Ex = a.E[0], *Ey = a.E[1], *Ez = a.E[2];
    T ex, ey, ez, bx, by, bz;
    {
        // every stencil below lies in the 4 x 4 nodes from (ic - 1, jc - 1)
        // around the particle's cell: their wrapped columns and row offsets
        // are formed once
        const int ic = (int)floor(x0 / dx), jc = (int)floor(y0 / dy);
        unsigned cw[4], rw[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            cw[k] = (unsigned)wrapc(ic - 1 + k, nx);
            rw[k] = (unsigned)wrapc(jc - 1 + k, ny) * (unsigned)nx;
        }
        auto pick = [](const unsigned (&w)[4], int k) { return k <= 0 ? w[0] : (k == 1 ? w[1] : (k == 2 ? w[2] : w[3])); };
        // value of a field at the particle: linear shapes around the
        // component's staggered position (i + ox, j + oy), the stencil's
        // nodes i0..i0+1 x j0..j0+1; val(col, row, c, b) reads node
        // (i0 + c, j0 + b) (columns col[c..c+1], rows row[b..b+1] for the
        // differences of the half Faraday step)
        auto gatherw = [&](auto &&val, T ox, T oy) {
            const T xi = x0 / dx - ox, eta = y0 / dy - oy;
            const int i0 = (int)floor(xi), j0 = (int)floor(eta);
            const int si = i0 - ic + 1, sj = j0 - jc + 1;
            const unsigned col[3] = {pick(cw, si), pick(cw, si + 1), pick(cw, si + 2)};
            const unsigned row[3] = {pick(rw, sj), pick(rw, sj + 1), pick(rw, sj + 2)};
            T v = T(0);
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    const T wgt = shape1(xi - T(i0 + c)) * shape1(eta - T(j0 + b));
                    v += wgt * val(col, row, c, b);
                }
            return v;
        };
        using U3 = const unsigned (&)[3];
        ex = gatherw([&](U3 cl, U3 rw_, int c, int b) { return Ex[rw_[b] + cl[c]]; }, T(0.5), T(0));
        ey = gatherw([&](U3 cl, U3 rw_, int c, int b) { return Ey[rw_[b] + cl[c]]; }, T(0), T(0.5));
        ez = gatherw([&](U3 cl, U3 rw_, int c, int b) { return Ez[rw_[b] + cl[c]]; }, T(0), T(0));
        // B^n at the B positions: half a Faraday step (eqs faraday_*, 2D)
        bx = gatherw([&](U3 cl, U3 rw_, int c, int b) {
            const T dyEz = (Ez[rw_[b + 1] + cl[c]] - Ez[rw_[b] + cl[c]]) / dy;
            return a.B[0][rw_[b] + cl[c]] - th * (dyEz - T(0));
        }, T(0), T(0.5));
        by = gatherw([&](U3 cl, U3 rw_, int c, int b) {
            const T dxEz = (Ez[rw_[b] + cl[c + 1]] - Ez[rw_[b] + cl[c]]) / dx;
            return a.B[1][rw_[b] + cl[c]] - th * (T(0) - dxEz);
        }, T(0.5), T(0));
        bz = gatherw([&](U3 cl, U3 rw_, int c, int b) {
            const T dxEy = (Ey[rw_[b] + cl[c + 1]] - Ey[rw_[b] + cl[c]]) / dx;
            const T dyEx = (Ex[rw_[b + 1] + cl[c]] - Ex[rw_[b] + cl[c]]) / dy;
            return a.B[2][rw_[b] + cl[c]] - th * (dxEy - dyEx);
        }, T(0.5), T(0.5));
    }
    // Boris: half electric kick, rotation about B, half electric kick
    const T h = a.h;
    const T umx = (live ? a.ux[p] : T(0)) + h * ex, umy = (live ? a.uy[p] : T(0)) + h * ey,
            umz = (live ? a.uz[p] : T(0)) + h * ez;
    const T gm = sqrt(T(1) + umx * umx + umy * umy + umz * umz);
    const T tx = h * bx / gm, ty = h * by / gm, tz = h * bz / gm;
    const T upx = umx + (umy * tz - umz * ty);
    const T upy = umy + (umz * tx - umx * tz);
    const T upz = umz + (umx * ty - umy * tx);
    const T f = T(2) / (T(1) + tx * tx + ty * ty + tz * tz);
    const T sx = f * tx, sy = f * ty, sz = f * tz;
    const T uplx = umx + (upy * sz - upz * sy);
    const T uply = umy + (upz * sx - upx * sz);
    const T uplz = umz + (upx * sy - upy * sx);
    const T nux = uplx + h * ex, nuy = uply + h * ey, nuz = uplz + h * ez;
    const T g = sqrt(T(1) + nux * nux + nuy * nuy + nuz * nuz);
    const T x1 = x0 + dt * nux / g, y1 = y0 + dt * nuy / g;
    // Esirkepov: shapes of the start and end positions on the window of
    // nodes i0 .. i0 + 3, j0 .. j0 + 3
    const T xi0 = x0 / dx, eta0 = y0 / dy, xi1 = x1 / dx, eta1 = y1 / dy;
    const int i0 = (int)floor(xi0) - 1, j0 = (int)floor(eta0) - 1;
    T sx0[4], sx1[4], sy0[4], sy1[4];
    for (int k = 0; k < 4; k++) {
        sx0[k] = shape1(xi0 - T(i0 + k));
        sx1[k] = shape1(xi1 - T(i0 + k));
        sy0[k] = shape1(eta0 - T(j0 + k));
        sy1[k] = shape1(eta1 - T(j0 + k));
    }
    const T vz = nuz / g;
    // the workgroup's windows: when they fit one LDS tile (particles kept in
    // cell order), the contributions are summed in LDS and added to J once
    // per node; otherwise each goes to J directly
    int imin = live ? i0 : 0x7fffffff, imax = live ? i0 : -0x7fffffff;
    block_minmax(imin, imax, sh);
    int jmin = live ? j0 : 0x7fffffff, jmax = live ? j0 : -0x7fffffff;
    block_minmax(jmin, jmax, sh);
    const int bw = imax + 4 - imin, bh = jmax + 4 - jmin;
    const bool in_lds = imax >= imin && bw <= TWX && bh <= TWY;
    if (in_lds) {
        for (int e = threadIdx.x; e < 3 * TPC; e += PT) tile[e] = T(0);
        __syncthreads();
    }
    // contribution e of the window: J_x at (k, l) = (e % 3, e / 3) for
    // e < 12, J_y at (k, l) = ((e - 12) / 3, (e - 12) % 3) for e < 24, J_z at
    // (k, l) = ((e - 24) % 4, (e - 24) / 4)
    auto node = [](int e, int &comp, int &k, int &l) {
        if (e < 12) { comp = 0; k = e % 3; l = e / 3; }
        else if (e < 24) { comp = 1; k = (e - 12) / 3; l = (e - 12) % 3; }
        else { comp = 2; k = (e - 24) % 4; l = (e - 24) / 4; }
    };
    T con[NCON];
#pragma unroll
    for (int l = 0; l < 4; l++) {
        T run = T(0);   // sum of W_x over the window's nodes up to k
        for (int k = 0; k < 3; k++) {
            run += T(0.5) * (sx1[k] - sx0[k]) * (sy0[l] + sy1[l]);
            con[3 * l + k] = a.cx * run;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        T run = T(0);   // sum of W_y over the window's nodes up to l
        for (int l = 0; l < 3; l++) {
            run += T(0.5) * (sy1[l] - sy0[l]) * (sx0[k] + sx1[k]);
            con[12 + 3 * k + l] = a.cy * run;
        }
    }
#pragma unroll
    for (int l = 0; l < 4; l++)
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const T wz = (T(2) * sx0[k] * sy0[l] + sx1[k] * sy0[l] + sx0[k] * sy1[l] + T(2) * sx1[k] * sy1[l]) / T(6);
            con[24 + 4 * l + k] = a.cz * vz * wz;
        }
    if (in_lds) {
        if (live)
#pragma unroll
            for (int e = 0; e < NCON; e++) {
                if (con[e] == T(0)) continue;
                int comp, k, l;
                node(e, comp, k, l);
                atomicAdd(&tile[comp * TPC + (j0 + l - jmin) * TPX + (i0 + k - imin)], con[e]);
            }
    } else if (live) {
#pragma unroll
        for (int e = 0; e < NCON; e++) {
            if (con[e] == T(0)) continue;
            int comp, k, l;
            node(e, comp, k, l);
            unsafeAtomicAdd(&a.J[comp][(size_t)wrapc(j0 + l, ny) * nx + wrapc(i0 + k, nx)], con[e]);
        }
    }
    if (live) {
        a.x[p] = x1 >= a.Lx ? x1 - a.Lx : (x1 < T(0) ? x1 + a.Lx : x1);
        a.y[p] = y1 >= a.Ly ? y1 - a.Ly : (y1 < T(0) ? y1 + a.Ly : y1);
        a.ux[p] = nux;
        a.uy[p] = nuy;
        a.uz[p] = nuz;
    }
    if (in_lds) {
        __syncthreads();
        for (int e = threadIdx.x; e < 3 * bw * bh; e += PT) {
            const int c = e / (bw * bh), r = e % (bw * bh);
            const T v = tile[c * TPC + (r / bw) * TPX + r % bw];
            if (v != T(0))
                unsafeAtomicAdd(&a.J[c][(size_t)wrapc(jmin + r / bw, ny) * nx + wrapc(imin + r % bw, nx)], v);
        }
    }
}

// rho at the nodes += q w / (dx dy) S(x/dx - i) S(y/dy - j)
template <typename T>
__global__ __launch_bounds__(PT) void k_pic_charge(int64_t np, int nx, int ny, T dx, T dy, T cq, const T *x,
                                                   const T *y, T *rho)
{
    const int64_t p = (int64_t)blockIdx.x * PT + threadIdx.x;
    if (p >= np) return;
    const T xi = x[p] / dx, eta = y[p] / dy;
    const int i0 = (int)floor(xi), j0 = (int)floor(eta);
    for (int b = 0; b < 2; b++)
        for (int c = 0; c < 2; c++) {
            const T v = cq * shape1(xi - T(i0 + c)) * shape1(eta - T(j0 + b));
            if (v != T(0)) unsafeAtomicAdd(&rho[(size_t)wrapn(j0 + b, ny) * nx + wrapn(i0 + c, nx)], v);
        }
}

template <typename T>
__global__ __launch_bounds__(PT) void k_fill0(int64_t n, T *a, T *b, T *c)
{
    const int64_t i = (int64_t)blockIdx.x * PT + threadIdx.x;
    if (i >= n) return;
    a[i] = T(0);
    if (b) b[i] = T(0);
    if (c) c[i] = T(0);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + PT - 1) / PT); }

}  // namespace

template <typename T>
hipError_t launch_pic_push(const PicArgs<T> &a, bool zero_j, hipStream_t s)
{
    const int64_t ncell = (int64_t)a.nx * a.ny;
    if (zero_j && ncell > 0)
        hipLaunchKernelGGL((k_fill0<T>), dim3(blocks_for(ncell)), dim3(PT), 0, s, ncell, a.J[0], a.J[1], a.J[2]);
    if (a.np > 0) hipLaunchKernelGGL((k_pic_push<T>), dim3(blocks_for(a.np)), dim3(PT), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pic_charge(int64_t np, int nx, int ny, T dx, T dy, T cq, const T *x, const T *y, T *rho,
                             bool zero_rho, hipStream_t s)
{
    const int64_t ncell = (int64_t)nx * ny;
    if (zero_rho && ncell > 0)
        hipLaunchKernelGGL((k_fill0<T>), dim3(blocks_for(ncell)), dim3(PT), 0, s, ncell, rho, (T *)nullptr,
                           (T *)nullptr);
    if (np > 0) hipLaunchKernelGGL((k_pic_charge<T>), dim3(blocks_for(np)), dim3(PT), 0, s, np, nx, ny, dx, dy, cq, x, y, rho);
    return hipGetLastError();
}

template hipError_t launch_pic_push<float>(const PicArgs<float> &, bool, hipStream_t);
template hipError_t launch_pic_push<double>(const PicArgs<double> &, bool, hipStream_t);
template hipError_t launch_pic_charge<float>(int64_t, int, int, float, float, float, const float *, const float *,
                                             float *, bool, hipStream_t);
template hipError_t launch_pic_charge<double>(int64_t, int, int, double, double, double, const double *,
                                              const double *, double *, bool, hipStream_t);

}  // namespace mx
