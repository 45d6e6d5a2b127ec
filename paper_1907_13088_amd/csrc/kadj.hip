// Kernels of the transposed (adjoint) step and of the localised 2D source
// shapes.  The forward step is linear in (E, B, J0):
//   B+ = B - dt K E,   E+ = E + P (dt K^T Lambda B+ - 4 pi dt env F J0)
// (eqs faraday_*, ampere_aux_*, transform-e-e_aux, Alg 1), with K the E->B
// curl, K^T the B->E curl, Lambda = diag(alpha_x, alpha_y, alpha_z) on B and
// F the binomial current filter.  A (Appendix C), Lambda and F are
// symmetric, so the transposed step is
//   v = P Ebar;  Bbar += dt Lambda K v;  J0bar += env (-4 pi dt) F v;
//   Ebar -= dt K^T Bbar.
// The sweeps for v reuse the forward sweep kernels; this file holds the
// curls, the filter of v and the source shapes.
#include "mx_internal.h"

namespace mx {
namespace {

constexpr int NT = 256;
constexpr int BXT = 64, BYT = 4;

__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

struct Ix {
    int nx, ny, nz, i, j, k;
    __device__ __forceinline__ size_t at(int di, int dj, int dk) const
    {
        return ((size_t)wrap1(k + dk, nz) * ny + wrap1(j + dj, ny)) * nx + wrap1(i + di, nx);
    }
};

__device__ __forceinline__ bool cell(int nx, int ny, Ix &id)
{
    id.i = blockIdx.x * BXT + (threadIdx.x & (BXT - 1));
    id.j = blockIdx.y * BYT + threadIdx.x / BXT;
    id.k = blockIdx.z;
    return id.i < nx && id.j < ny;
}

template <typename T>
__device__ __forceinline__ T avg(T fm, T f0, T fp, int lumped)
{
    return lumped ? f0 : f0 + (fm + fp - T(2) * f0) * T(1.0 / 6.0);
}

// Bbar += dt Lambda K v.  dt (K v) at B positions:
//   x: tdy (vz[j+1] - vz) - tdz (vy[k+1] - vy)
//   y: tdz (vx[k+1] - vx) - tdx (vz[i+1] - vz)
//   z: tdx (vy[i+1] - vy) - tdy (vx[j+1] - vx)
// and, when acc is set, acc += sc v on the stepped components (the current
// gradient's accumulator, the same axpy as k_axpy, while v is at hand)
template <typename T>
__global__ __launch_bounds__(NT) void k_adj_curlB(Coef<T> c, int ndim, int blocks, const T *vx,
                                                  const T *vy, const T *vz, T *Bx, T *By, T *Bz, T sc, T *ax,
                                                  T *ay, T *az)
{
    Ix id{c.nx, c.ny, c.nz, 0, 0, 0};
    if (!cell(c.nx, c.ny, id)) return;
    const bool d3 = ndim == 3;
    const bool te = d3 || (blocks & 1), tm = d3 || (blocks & 2);
    auto kx = [&](int di, int dj, int dk) {
        T r = c.tdy * (vz[id.at(di, dj + 1, dk)] - vz[id.at(di, dj, dk)]);
        if (d3) r -= c.tdz * (vy[id.at(di, dj, dk + 1)] - vy[id.at(di, dj, dk)]);
        return r;
    };
    auto ky = [&](int di, int dj, int dk) {
        T r = -c.tdx * (vz[id.at(di + 1, dj, dk)] - vz[id.at(di, dj, dk)]);
        if (d3) r += c.tdz * (vx[id.at(di, dj, dk + 1)] - vx[id.at(di, dj, dk)]);
        return r;
    };
    auto kz = [&](int di, int dj, int dk) {
        return c.tdx * (vy[id.at(di + 1, dj, dk)] - vy[id.at(di, dj, dk)])
             - c.tdy * (vx[id.at(di, dj + 1, dk)] - vx[id.at(di, dj, dk)]);
    };
    const size_t o = id.at(0, 0, 0);
    const int L = c.lumped;
    if (tm) {
        Bx[o] += avg(kx(-1, 0, 0), kx(0, 0, 0), kx(1, 0, 0), L);
        By[o] += avg(ky(0, -1, 0), ky(0, 0, 0), ky(0, 1, 0), L);
    }
    if (te) Bz[o] += d3 ? avg(kz(0, 0, -1), kz(0, 0, 0), kz(0, 0, 1), L) : kz(0, 0, 0);
    if (ax) {
        if (te) {
            ax[o] += sc * vx[o];
            ay[o] += sc * vy[o];
        }
        if (tm) az[o] += sc * vz[o];
    }
}

// Ebar -= dt K^T Bbar (the B->E curl of the auxiliary equations, Lambda = 1)
template <typename T>
__global__ __launch_bounds__(NT) void k_adj_curlE(Coef<T> c, int ndim, int blocks, const T *Bx,
                                                  const T *By, const T *Bz, T *Ex, T *Ey, T *Ez)
{
    Ix id{c.nx, c.ny, c.nz, 0, 0, 0};
    if (!cell(c.nx, c.ny, id)) return;
    const bool d3 = ndim == 3;
    const bool te = d3 || (blocks & 1), tm = d3 || (blocks & 2);
    const size_t o = id.at(0, 0, 0);
    if (te) {
        T cx = c.tdy * (Bz[o] - Bz[id.at(0, -1, 0)]);
        T cy = -c.tdx * (Bz[o] - Bz[id.at(-1, 0, 0)]);
        if (d3) {
            cx -= c.tdz * (By[o] - By[id.at(0, 0, -1)]);
            cy += c.tdz * (Bx[o] - Bx[id.at(0, 0, -1)]);
        }
        Ex[o] -= cx;
        Ey[o] -= cy;
    }
    if (tm) Ez[o] -= c.tdx * (By[o] - By[id.at(-1, 0, 0)]) - c.tdy * (Bx[o] - Bx[id.at(0, -1, 0)]);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_filter_axis(Coef<T> c, int axis, const T *src, T *dst)
{
    Ix id{c.nx, c.ny, c.nz, 0, 0, 0};
    if (!cell(c.nx, c.ny, id)) return;
    const int di = axis == 0, dj = axis == 1, dk = axis == 2;
    dst[id.at(0, 0, 0)] = T(0.25) * src[id.at(-di, -dj, -dk)] + T(0.5) * src[id.at(0, 0, 0)]
                        + T(0.25) * src[id.at(di, dj, dk)];
}

template <typename T>
__global__ __launch_bounds__(NT) void k_axpy(int64_t n, T a, const T *x, T *y)
{
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}

template <typename T>
__global__ __launch_bounds__(NT) void k_fill(int64_t n, T *y)
{
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) y[i] = T(0);
}

__device__ __forceinline__ int cyc(int64_t v, int n)
{
    const int64_t r = v % n;
    return (int)(r < 0 ? r + n : r);
}

// J0 = sum_s amps[s] shape_s (J0 overwritten).  A workgroup owns a BXT x BYT
// block of cells, one per thread: it lists, in source order, the sources
// whose (periodically wrapped) windows reach the block and adds them to its
// cells' sums in that order, so every cell sums its contributions in source
// order whatever the launch (0 + the first, then each next one).
template <typename T>
__global__ __launch_bounds__(NT) void k_src_assemble(int nx, int ny, int nsrc, int W, const int64_t *org,
                                                     const T *shapes, const T *amps, T *Jx, T *Jy, T *Jz)
{
    __shared__ int list[NT];
    __shared__ int wsum[NT / 64];
    T *J[3] = {Jx, Jy, Jz};
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int bx0 = blockIdx.x * BXT, by0 = blockIdx.y * BYT;
    const int bw = min(BXT, nx - bx0), bh = min(BYT, ny - by0);
    const int i = bx0 + (tid & (BXT - 1)), j = by0 + tid / BXT;
    const bool own = i < nx && j < ny;
    T acc[3] = {T(0), T(0), T(0)};
    for (int c0 = 0; c0 < nsrc; c0 += NT) {
        // does source c0 + tid reach the block?  (cyclic intervals intersect
        // when either start lies inside the other interval)
        const int s = c0 + tid;
        bool hit = false;
        if (s < nsrc) {
            const int xs = cyc(org[2 * s], nx), ys = cyc(org[2 * s + 1], ny);
            hit = (cyc((int64_t)bx0 - xs, nx) < W || cyc((int64_t)xs - bx0, nx) < bw) &&
                  (cyc((int64_t)by0 - ys, ny) < W || cyc((int64_t)ys - by0, ny) < bh);
        }
        // ordered compaction of the hits into list[]
        const unsigned long long m = __ballot(hit);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wv] = __popcll(m);
        __syncthreads();
        int base = 0, total = 0;
        for (int w = 0; w < NT / 64; w++) {
            if (w < wv) base += wsum[w];
            total += wsum[w];
        }
        if (hit) list[base + before] = s;
        __syncthreads();
        if (own)
            for (int e = 0; e < total; e++) {
                const int sr = list[e];
                const int bb = cyc((int64_t)i - org[2 * sr], nx), aa = cyc((int64_t)j - org[2 * sr + 1], ny);
                if (bb >= W || aa >= W) continue;
                const T a = amps[sr];
                for (int q = 0; q < 3; q++) acc[q] += a * shapes[((size_t)(sr * 3 + q) * W + aa) * W + bb];
            }
        __syncthreads();   // list[] and wsum[] are reused by the next chunk
    }
    if (own)
        for (int q = 0; q < 3; q++) J[q][(size_t)j * nx + i] = acc[q];
}

// grad[s] = <shape_s, G>, one workgroup per source, fixed-order reduction
template <typename T>
__global__ __launch_bounds__(NT) void k_src_project(int nx, int ny, int W, const int64_t *org,
                                                    const T *shapes, const T *Gx, const T *Gy,
                                                    const T *Gz, T *grad)
{
    __shared__ double sh[NT];
    const T *G[3] = {Gx, Gy, Gz};
    const int s = blockIdx.x;
    const int64_t x0 = org[2 * s], y0 = org[2 * s + 1];
    double acc = 0.0;
    for (int t = threadIdx.x; t < W * W; t += NT) {
        const int aa = t / W, bb = t - aa * W;
        const size_t o = (size_t)(((y0 + aa) % ny + ny) % ny) * nx + (size_t)(((x0 + bb) % nx + nx) % nx);
        for (int q = 0; q < 3; q++)
            acc += (double)shapes[((size_t)(s * 3 + q) * W + aa) * W + bb] * (double)G[q][o];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[s] = (T)sh[0];
}

dim3 grid3(int nx, int ny, int nz) { return dim3((nx + BXT - 1) / BXT, (ny + BYT - 1) / BYT, nz); }

}  // namespace

template <typename T>
hipError_t launch_adj_curlB(const Coef<T> &c, int ndim, int blocks, const T *const v[3],
                            T *const Bbar[3], T sc, T *const acc[3], hipStream_t s)
{
    hipLaunchKernelGGL((k_adj_curlB<T>), grid3(c.nx, c.ny, c.nz), dim3(NT), 0, s, c, ndim, blocks,
                       v[0], v[1], v[2], Bbar[0], Bbar[1], Bbar[2], sc, acc ? acc[0] : nullptr,
                       acc ? acc[1] : nullptr, acc ? acc[2] : nullptr);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_curlE(const Coef<T> &c, int ndim, int blocks, const T *const Bbar[3],
                            T *const Ebar[3], hipStream_t s)
{
    hipLaunchKernelGGL((k_adj_curlE<T>), grid3(c.nx, c.ny, c.nz), dim3(NT), 0, s, c, ndim, blocks,
                       Bbar[0], Bbar[1], Bbar[2], Ebar[0], Ebar[1], Ebar[2]);
    return hipGetLastError();
}

// dJ0 += scale * F v (F = p passes of (1,2,1)/4 per axis)
template <typename T>
hipError_t launch_adj_source(const Coef<T> &c, int ndim, int passes, const T *const v[3],
                             T *const tmp1[3], T *const tmp2[3], T scale, T *const dJ0[3],
                             hipStream_t s)
{
    const int64_t n = (int64_t)c.nx * c.ny * c.nz;
    const unsigned nb = (unsigned)((n + NT - 1) / NT);
    for (int q = 0; q < 3; q++) {
        const T *src = v[q];
        const int total = ndim * passes;
        for (int t = 0; t < total; t++) {
            T *dst = (t % 2 == 0) ? tmp1[q] : tmp2[q];
            hipLaunchKernelGGL((k_filter_axis<T>), grid3(c.nx, c.ny, c.nz), dim3(NT), 0, s, c, t % ndim, src, dst);
            src = dst;
        }
        hipLaunchKernelGGL((k_axpy<T>), dim3(nb), dim3(NT), 0, s, n, scale, src, dJ0[q]);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sources(int nx, int ny, int nsrc, int W, const int64_t *origins, const T *shapes,
                          const T *amps, T *const J0[3], T *const G[3], T *grad, bool project,
                          hipStream_t s)
{
    if (!project) {
        hipLaunchKernelGGL((k_src_assemble<T>), grid3(nx, ny, 1), dim3(NT), 0, s, nx, ny, nsrc, W, origins, shapes,
                           amps, J0[0], J0[1], J0[2]);
    } else {
        hipLaunchKernelGGL((k_src_project<T>), dim3(nsrc), dim3(NT), 0, s, nx, ny, W, origins, shapes,
                           G[0], G[1], G[2], grad);
    }
    return hipGetLastError();
}

// acc[q] = 0 (zero != 0) or acc[q] += a x[q], for the components in mask
template <typename T>
hipError_t launch_axpy3(int64_t n, int mask, bool zero, T a, const T *const x[3], T *const acc[3], hipStream_t s)
{
    const unsigned nb = (unsigned)((n + NT - 1) / NT);
    for (int q = 0; q < 3; q++) {
        if (!(mask & (1 << q))) continue;
        if (zero) hipLaunchKernelGGL((k_fill<T>), dim3(nb), dim3(NT), 0, s, n, acc[q]);
        else hipLaunchKernelGGL((k_axpy<T>), dim3(nb), dim3(NT), 0, s, n, a, x[q], acc[q]);
    }
    return hipGetLastError();
}

#define INST(T)                                                                                       \
    template hipError_t launch_adj_curlB<T>(const Coef<T> &, int, int, const T *const[3], T *const[3], \
                                            T, T *const[3], hipStream_t);                             \
    template hipError_t launch_adj_curlE<T>(const Coef<T> &, int, int, const T *const[3], T *const[3], \
                                            hipStream_t);                                             \
    template hipError_t launch_adj_source<T>(const Coef<T> &, int, int, const T *const[3], T *const[3], \
                                             T *const[3], T, T *const[3], hipStream_t);               \
    template hipError_t launch_sources<T>(int, int, int, int, const int64_t *, const T *, const T *,  \
                                          T *const[3], T *const[3], T *, bool, hipStream_t);           \
    template hipError_t launch_axpy3<T>(int64_t, int, bool, T, const T *const[3], T *const[3], hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace mx
