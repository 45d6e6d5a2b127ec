// 3D kernels of the field step (arXiv 1907.13088, Sec. 2.2.1) for filters
// of more than two passes (the fused front, k3f.hip, covers up to two):
//   Faraday update ........ eqs faraday_x..z
//   current filter ........ p passes of (1,2,1)/4 along x, y and z
//   auxiliary increment ... eqs ampere_aux_x..z
// One thread per cell, 64 x 4 threads per workgroup along x and y, one z
// plane per workgroup row of the grid; neighbour values come through the
// vector caches.  The sweep passes are in k3s.hip.
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
    return launch_stream3d<T>(c, k, form, flags, a, s, nwg);
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
