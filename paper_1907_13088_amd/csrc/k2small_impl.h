#pragma once
// Single-launch tolerance solve for small 2D grids (Alg. 1 with the stop
// test of each block, Sec. 2.2.1): grids too small to fill the GPU with
// row streams spend most of a step in launch gaps (front, one sweep pass,
// reduction and stop test per pass, E increment).  Here one cooperative
// launch runs up to SMALL_MAX_STEPS whole steps: per step the front (Faraday,
// filter of the current, auxiliary increment dE' and its FP64 norm) on each
// workgroup's tile with a recomputed halo, then passes of the LDS-tile sweep
// (the same device function as the per-launch kernel, so the iterates are
// bitwise those of a replay of the same counts), each followed by the FP64
// reduction of the per-workgroup norms, which every workgroup sums in the
// same order and so takes the same stop decision, then the E increment.
// Phases are separated by the bounded grid barrier; workgroup 0 records
// each step's counts and norms.
#include "gridbar.h"
#include "k2tile.h"

namespace mx {
namespace small2d {

// Tile shape and threads per workgroup: FP64 512 threads on a 32 x 8 tile
// (a pass of 8 sweeps covers a 48 x 24 region, 2.25 cells per thread), FP32
// 1024 threads on 32 x 16.  128^2 FP64 tolerance solve, medians of five
// runs of 1000 steps on one box: 32 x 8 tiles with 512 threads 56.7 us per
// step, 384 threads 59.1, 768 threads 58.5, 1024 threads 61.3; 32 x 4 tiles
// 69.2 (512 threads) and 68.6 (1024), 16 x 8 tiles 63.9 and 65.7, 16 x 4
// tiles 88.5, 32 x 16 tiles of 1024 threads 62.9 (earlier, with every pass
// depth unrolled: 104 us per step with 256 threads, against 98 with 1024)
template <typename T> struct Tile;
template <> struct Tile<double> { static constexpr int TX = 32, TY = 8, NT = 512; };
template <> struct Tile<float> { static constexpr int TX = 32, TY = 16, NT = 1024; };
constexpr int PMAX = 4;   // filter passes
constexpr int KMAX = 8;   // sweeps per pass

template <typename T>
constexpr size_t front_bytes()
{
    constexpr int TX = Tile<T>::TX, TY = Tile<T>::TY;
    return sizeof(T) * (3 * (TX + 3) * (TY + 3) + 3 * (TX + 2) * (TY + 2) + 3 * (TX + 2 * PMAX) * (TY + 2 * PMAX) +
                        3 * TX * (TY + 2 * PMAX));
}
template <typename T>
constexpr size_t lds_bytes()
{
    constexpr size_t sw = tile2d::sweep_lds_bytes<T, 3, KMAX, Tile<T>::TX, Tile<T>::TY>();
    return sw > front_bytes<T>() ? sw : front_bytes<T>();
}

// Element i of a global array whose pointer is chosen at run time from a
// small local table (the previous step's increment): read as a global load
// (through the table the compiler would emit a flat one)
template <typename T>
__device__ __forceinline__ T ld_at(const T *p, size_t i)
{
    return *(gptr<const T>)(p + i);
}

// the filter's x weights: binomial(2P, t) / 4^P
template <int P>
__device__ __forceinline__ constexpr float binom(int t)
{
    float c = 1.0f;
    for (int i = 0; i < t; i++) c = c * (float)(2 * P - i) / (float)(i + 1);
    float d = 1.0f;
    for (int i = 0; i < P; i++) d *= 4.0f;
    return c / d;
}

// alpha f = f + (f- + f+ - 2 f)/6 (sixth = 0: the lumped scheme)
template <typename T>
__device__ __forceinline__ T avg6(T fm, T f0, T fp, T sixth)
{
    return fma(fma(T(-2), f0, fm + fp), sixth, f0);
}

// The front of step s on tile (bx, by): B^{n+1/2} on the tile and a
// one-cell halo, dE' on the tile, its FP64 norm per block in partial[wg].
// The arithmetic of each output is that of the streaming front kernel.
// inc[q] (null: none) is the previous step's increment of E component q,
// not yet added to E in memory: E^n = E + inc, formed as the E update forms it.
template <typename T, int P>
__device__ __forceinline__ void front(const SmallArgs<T> &a, int s, int bx, int by, int wg, char *lds, double *sred,
                                      const T *const inc[3])
{
    constexpr int TX = Tile<T>::TX, TY = Tile<T>::TY, NT = Tile<T>::NT;
    constexpr int EX = TX + 3, EY = TY + 3, BX = TX + 2, BY = TY + 2, JX = TX + 2 * P, JY = TY + 2 * P;
    T(*sE)[EY][EX] = reinterpret_cast<T(*)[EY][EX]>(lds);
    T(*sB)[BY][BX] = reinterpret_cast<T(*)[BY][BX]>(lds + sizeof(T) * 3 * EY * EX);
    T(*sJ)[JY][JX] = reinterpret_cast<T(*)[JY][JX]>(lds + sizeof(T) * 3 * (EY * EX + BY * BX));
    T(*sJx)[JY][TX] = reinterpret_cast<T(*)[JY][TX]>(lds + sizeof(T) * 3 * (EY * EX + BY * BX + JY * JX));
    const Coef<T> &c = a.c;
    const int nx = c.nx, ny = c.ny, tid = threadIdx.x;
    const int X0 = bx * TX, Y0 = by * TY;
    const bool TE = a.blocks & 1, TM = a.blocks & 2;
    const bool hasj = a.J0[0] != nullptr;
    const T sixth = c.lumped ? T(0) : T(1.0 / 6.0);
    const T es = a.env_src[s];
    using tile2d::wrapi;
    const T *Bin[3];
    T *Bout[3];
    for (int q = 0; q < 3; q++) {
        // parity selects without indexing the argument block at run time
        Bin[q] = (s & 1) ? a.B[1][q] : a.B[0][q];
        Bout[q] = (s & 1) ? a.B[0][q] : a.B[1][q];
    }
    for (int e = tid; e < 3 * EY * EX; e += NT) {
        const int q = e / (EY * EX), r = e % (EY * EX), iy = r / EX, ix = r % EX;
        if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
        const size_t o = (size_t)wrapi(Y0 - 1 + iy, ny) * nx + wrapi(X0 - 1 + ix, nx);
        const T *iq = q == 0 ? inc[0] : (q == 1 ? inc[1] : inc[2]);
        sE[q][iy][ix] = iq ? a.E[q][o] + ld_at(iq, o) : a.E[q][o];
    }
    if (hasj)
        for (int e = tid; e < 3 * JY * JX; e += NT) {
            const int q = e / (JY * JX), r = e % (JY * JX), iy = r / JX, ix = r % JX;
            if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
            sJ[q][iy][ix] = a.J0[q][(size_t)wrapi(Y0 - P + iy, ny) * nx + wrapi(X0 - P + ix, nx)];
        }
    __syncthreads();
    // B^{n+1/2} = B^{n-1/2} - dt curl E^n on the tile and its halo (the E
    // tile's cell (ix, iy) is the B region's cell (ix, iy))
    for (int e = tid; e < BY * BX; e += NT) {
        const int iy = e / BX, ix = e % BX;
        const int gx = X0 - 1 + ix, gy = Y0 - 1 + iy;
        const size_t o = (size_t)wrapi(gy, ny) * nx + wrapi(gx, nx);
        const bool own = ix >= 1 && ix <= TX && iy >= 1 && iy <= TY && gx < nx && gy < ny;
        if (TM) {
            const T ez = sE[2][iy][ix];
            const T bxv = Bin[0][o] - c.tdy * (sE[2][iy + 1][ix] - ez);
            const T byv = Bin[1][o] + c.tdx * (sE[2][iy][ix + 1] - ez);
            sB[0][iy][ix] = bxv;
            sB[1][iy][ix] = byv;
            if (own) { Bout[0][o] = bxv; Bout[1][o] = byv; }
        }
        if (TE) {
            const T bzv = Bin[2][o] - (c.tdx * (sE[1][iy][ix + 1] - sE[1][iy][ix]) -
                                       c.tdy * (sE[0][iy + 1][ix] - sE[0][iy][ix]));
            sB[2][iy][ix] = bzv;
            if (own) Bout[2][o] = bzv;
        }
    }
    // x filter of the current rows: (2P + 1) binomial taps
    if (hasj)
        for (int e = tid; e < 3 * JY * TX; e += NT) {
            const int q = e / (JY * TX), r = e % (JY * TX), y = r / TX, x = r % TX;
            if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
            T v = T(0);
            for (int k = -P; k <= P; k++) v = fma(T(binom<P>(k + P)), sJ[q][y][x + P + k], v);
            sJx[q][y][x] = v;
        }
    __syncthreads();
    double nte = 0.0, ntm = 0.0;
    for (int e = tid; e < TX * TY; e += NT) {
        const int y = e / TX, x = e % TX;
        const int gx = X0 + x, gy = Y0 + y;
        if (gx >= nx || gy >= ny) continue;
        // y filter: P cascaded three-tap passes over the x-filtered rows
        T jf[3] = {T(0), T(0), T(0)};
        if (hasj)
            for (int q = 0; q < 3; q++) {
                if ((q < 2 && !TE) || (q == 2 && !TM)) continue;
                T w[2 * P + 1];
                for (int i = 0; i <= 2 * P; i++) w[i] = sJx[q][y + i][x];
                for (int r = 1; r <= P; r++)
                    for (int i = 0; i + 2 * r <= 2 * P; i++) w[i] = T(0.25) * fma(T(2), w[i + 1], w[i] + w[i + 2]);
                jf[q] = w[0];
            }
        const int cx = x + 1, cy = y + 1;
        const size_t o = (size_t)gy * nx + gx;
        if (TE) {
            const T vx = c.tdy * (sB[2][cy][cx] - sB[2][cy - 1][cx]) - es * jf[0];
            const T vy = -c.tdx * (sB[2][cy][cx] - sB[2][cy][cx - 1]) - es * jf[1];
            a.dEp[0][o] = vx;
            a.dEp[1][o] = vy;
            nte += (double)vx * vx + (double)vy * vy;
        }
        if (TM) {
            const T ay = avg6(sB[1][cy - 1][cx], sB[1][cy][cx], sB[1][cy + 1][cx], sixth);
            const T ayl = avg6(sB[1][cy - 1][cx - 1], sB[1][cy][cx - 1], sB[1][cy + 1][cx - 1], sixth);
            const T axj = avg6(sB[0][cy][cx - 1], sB[0][cy][cx], sB[0][cy][cx + 1], sixth);
            const T axm = avg6(sB[0][cy - 1][cx - 1], sB[0][cy - 1][cx], sB[0][cy - 1][cx + 1], sixth);
            const T vz = c.tdx * (ay - ayl) - c.tdy * (axj - axm) - es * jf[2];
            a.dEp[2][o] = vz;
            ntm += (double)vz * vz;
        }
    }
    tile2d::block_sum2<NT>(nte, ntm, sred);
    if (tid == 0) {
        a.partial[2 * wg] = nte;
        a.partial[2 * wg + 1] = ntm;
    }
}

// sum of the per-workgroup partials, the same in every workgroup
template <int NT>
__device__ __forceinline__ void reduce_partials(const double *partial, int nwg, double *sred, double *sdec,
                                                double &ra, double &rb)
{
    double x = 0.0, y = 0.0;
    for (int i = threadIdx.x; i < nwg; i += NT) {
        x += partial[2 * i];
        y += partial[2 * i + 1];
    }
    tile2d::block_sum2<NT>(x, y, sred);
    if (threadIdx.x == 0) { sdec[0] = x; sdec[1] = y; }
    __syncthreads();
    ra = sdec[0];
    rb = sdec[1];
    __syncthreads();
}

// A pass of k <= KMAX sweeps: one code path for every depth (a level loop
// over the region of KMAX), which keeps the kernel's registers those of one
// pass instead of eight inlined depths
template <typename T, int BLK, bool DELTA>
__device__ __forceinline__ void sweep_k(const Coef<T> &c, const SweepArgs<T> &sa, int flags, int k, int bx, int by, int wg,
                        char *lds, double *sred)
{
    constexpr int TX = Tile<T>::TX, TY = Tile<T>::TY, NT = Tile<T>::NT;
    tile2d::sweep_tile<T, BLK, KMAX, TX, TY, DELTA, NT, true>(c, sa, flags, bx, by, wg, lds, sred, k);
}

// E += inc on the own tile (inc[q] null: component unchanged)
template <typename T>
__device__ __forceinline__ void add_increment(const SmallArgs<T> &a, int bx, int by, const T *const inc[3])
{
    constexpr int TX = Tile<T>::TX, TY = Tile<T>::TY, NT = Tile<T>::NT;
    const int nx = a.c.nx, ny = a.c.ny;
    for (int e = threadIdx.x; e < TX * TY; e += NT) {
        const int gx = bx * TX + e % TX, gy = by * TY + e / TX;
        if (gx >= nx || gy >= ny) continue;
        const size_t o = (size_t)gy * nx + gx;
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const T *iq = q == 0 ? inc[0] : (q == 1 ? inc[1] : inc[2]);
            if (iq) a.E[q][o] += ld_at(iq, o);
        }
    }
}

// A step's E increment is added to E in memory after the next step's front
// has read E (the front adds it on the fly for its tile and halo), right
// after the barrier that ends that front and before the first sweep pass
// can overwrite the iterate: no barrier of its own.
// BLKS: the blocks the grid steps (1 TE, 2 TM, 3 both); a kernel holds the
// sweep variants of those blocks only (as the active blocks of a two-block
// grid change, 3 holds all three).
template <typename T, bool DELTA, int BLKS>
__global__ __launch_bounds__(Tile<T>::NT) void k2_small(SmallArgs<T> a)
{
    constexpr int NT = Tile<T>::NT;
    __shared__ __attribute__((aligned(16))) char lds[lds_bytes<T>()];
    __shared__ double sred[2 * NT / 64];
    __shared__ double sdec[2];
    __shared__ int sflag;
    const Coef<T> &c = a.c;
    const int nwg = gridDim.x;
    const int wg = xcd_map(blockIdx.x, nwg);   // tiles x-fastest, neighbours on one XCD
    const int bx = wg % a.ntx, by = wg / a.ntx;
    const T *inc[3] = {nullptr, nullptr, nullptr};   // the previous step's E increment
    for (int s = 0; s < a.nsteps; s++) {
        switch (a.filter_passes) {
        case 0: front<T, 0>(a, s, bx, by, wg, lds, sred, inc); break;
        case 1: front<T, 1>(a, s, bx, by, wg, lds, sred, inc); break;
        case 2: front<T, 2>(a, s, bx, by, wg, lds, sred, inc); break;
        case 3: front<T, 3>(a, s, bx, by, wg, lds, sred, inc); break;
        default: front<T, 4>(a, s, bx, by, wg, lds, sred, inc); break;
        }
        if (!grid_barrier(a.bar, nwg, a.err, &sflag)) return;
        add_increment(a, bx, by, inc);
        SmallStat st{};
        double r0, r1;
        reduce_partials<NT>(a.partial, nwg, sred, sdec, r0, r1);
        st.rhsn[0] = (a.blocks & 1) ? sqrt(r0) : 0.0;
        st.rhsn[1] = (a.blocks & 2) ? sqrt(r1) : 0.0;
        bool active[2];
        for (int b = 0; b < 2; b++) {
            if (!isfinite(st.rhsn[b])) st.nonfinite |= 1;
            // dE' = 0: the increment is 0, no sweeps
            active[b] = (a.blocks & (1 << b)) && st.rhsn[b] > 0.0 && isfinite(st.rhsn[b]);
        }
        int last[2] = {-1, -1}, cur = -1;
        while (!st.nonfinite && (active[0] || active[1])) {
            const int b0 = active[0] ? 0 : 1;
            const int kk = min(a.spp, a.mmax - st.done[b0]);
            const bool first = st.done[b0] == 0;
            const int ob = cur == 0 ? 1 : 0;
            SweepArgs<T> sa{};
            for (int q = 0; q < 3; q++) {
                sa.rhs[q] = a.dEp[q];
                sa.x_in[q] = first ? a.dEp[q] : (cur == 1 ? a.X[1][q] : a.X[0][q]);
                sa.s_in[q] = a.S[q];
                sa.x_out[q] = ob == 1 ? a.X[1][q] : a.X[0][q];
                sa.s_out[q] = a.S[q];
                sa.E[q] = a.E[q];
            }
            sa.partial = a.partial;
            const int flags = (first ? SW_FIRST : 0) | SW_RESID | SW_STORE;
            const int act = (active[0] ? 1 : 0) | (active[1] ? 2 : 0);
            if constexpr (BLKS == 1) {
                sweep_k<T, 1, DELTA>(c, sa, flags, kk, bx, by, wg, lds, sred);
            } else if constexpr (BLKS == 2) {
                sweep_k<T, 2, DELTA>(c, sa, flags, kk, bx, by, wg, lds, sred);
            } else {
                if (act == 1) sweep_k<T, 1, DELTA>(c, sa, flags, kk, bx, by, wg, lds, sred);
                else if (act == 2) sweep_k<T, 2, DELTA>(c, sa, flags, kk, bx, by, wg, lds, sred);
                else sweep_k<T, 3, DELTA>(c, sa, flags, kk, bx, by, wg, lds, sred);
            }
            if (!grid_barrier(a.bar, nwg, a.err, &sflag)) return;
            reduce_partials<NT>(a.partial, nwg, sred, sdec, r0, r1);
            const double r[2] = {sqrt(r0), sqrt(r1)};
            for (int b = 0; b < 2; b++) {
                if (!active[b]) continue;
                st.done[b] += kk;
                last[b] = ob;
                st.resid[b] = r[b];
                if (!isfinite(r[b])) {
                    st.nonfinite |= 2;
                    active[b] = false;
                } else if (r[b] <= a.tol * st.rhsn[b]) {
                    st.conv[b] = 1;
                    active[b] = false;
                } else if (st.done[b] >= a.mmax) {
                    active[b] = false;
                }
            }
            cur = ob;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) a.stat[s] = st;
        if (st.nonfinite) return;   // every workgroup took the same decision
        // this step's increment: dE = S (delta form) or the last iterate
        for (int q = 0; q < 3; q++) {
            const int b = q == 2 ? 1 : 0;
            const T *d = st.done[b] == 0 ? nullptr
                         : DELTA         ? (q == 0 ? a.S[0] : (q == 1 ? a.S[1] : a.S[2]))
                         : last[b] == 1  ? (q == 0 ? a.X[1][0] : (q == 1 ? a.X[1][1] : a.X[1][2]))
                                         : (q == 0 ? a.X[0][0] : (q == 1 ? a.X[0][1] : a.X[0][2]));
            if (q == 0) inc[0] = d;
            else if (q == 1) inc[1] = d;
            else inc[2] = d;
        }
    }
    // the last step's increment (no front follows within this launch)
    add_increment(a, bx, by, inc);
}

}  // namespace small2d

template <typename T>
void small_tiles(int nx, int ny, int *ntx, int *nty)
{
    *ntx = (nx + small2d::Tile<T>::TX - 1) / small2d::Tile<T>::TX;
    *nty = (ny + small2d::Tile<T>::TY - 1) / small2d::Tile<T>::TY;
}

namespace small2d {
template <typename T>
const void *kernel(bool delta, int blocks)
{
    if (delta)
        return blocks == 1 ? (const void *)k2_small<T, true, 1>
               : blocks == 2 ? (const void *)k2_small<T, true, 2> : (const void *)k2_small<T, true, 3>;
    return blocks == 1 ? (const void *)k2_small<T, false, 1>
           : blocks == 2 ? (const void *)k2_small<T, false, 2> : (const void *)k2_small<T, false, 3>;
}
}  // namespace small2d

template <typename T>
int small_capacity(bool delta, int blocks)
{
    static std::atomic<int> cache[2][3][MX_MAX_DEVICES];
    return per_device(cache[delta ? 1 : 0][blocks - 1], [&]() {
        int dev = 0, coop = 0, cu = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 0;
        if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        const void *k = small2d::kernel<T>(delta, blocks);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, small2d::Tile<T>::NT, 0) != hipSuccess) return 0;
        return per * cu;
    });
}

template <typename T>
hipError_t launch_small(const SmallArgs<T> &a, bool delta, hipStream_t s)
{
    void *args[] = {(void *)&a};
    const int nwg = a.ntx * a.nty;
    const void *k = small2d::kernel<T>(delta, a.blocks);
    return hipLaunchCooperativeKernel(k, dim3(nwg), dim3(small2d::Tile<T>::NT), args, 0, s);
}

}  // namespace mx
