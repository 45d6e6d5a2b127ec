// Fused 3D front pass of the field step (arXiv 1907.13088, Sec. 2.2.1):
//   Faraday update ........ B^{n+1/2} = B^{n-1/2} - dt curl E^n (eqs faraday_x..z)
//   current filter ........ p passes of (1,2,1)/4 along x, y and z (p <= 2)
//   auxiliary increment ... dE' = dt curl(Lambda B^{n+1/2}) - 4 pi dt env Jf
//                           (eqs ampere_aux_x..z)
// in one pass over HBM that reads E, B^{n-1/2} and J0 once and writes
// B^{n+1/2} (to the other B buffer) and dE'.
//
// A workgroup of FX x FY threads owns an FX x FY column tile and marches in z
// over a chunk of planes.  At march step t it stages plane t of E (tile plus
// x, y halo [-1, +2]) and plane t - 2 + p of the raw current (halo p) in LDS,
// computes B^{n+1/2} at plane t - 1 on the tile plus a one-cell halo (so the
// curl of Lambda B needs no neighbour's result: the halo is recomputed), and
// dE' at plane t - 2 from the three newest B^{n+1/2} planes.  The current is
// filtered along x and y in LDS and along z by p cascaded three-tap passes in
// registers, each thread for its own column.  Two barriers per plane.
#include <algorithm>

#include "mx_internal.h"

namespace mx {
namespace {

// Tile of FX x FY columns, one thread each: FP32 128 x 8 (1024 threads),
// FP64 64 x 8 (the LDS of a 1024-thread FP64 tile would exceed a CU's).
// 512^3 FP32, p = 1, one plane in flight: 128 x 8 took 1.98 ms per step
// against 2.10 with 64 x 16, 2.41 with 64 x 8 and 2.60 with 32 x 32: rows
// of 128 columns touch 6 cache lines for 4 useful ones (64 columns: 4 for
// 2), which outweighs the larger recomputed B^{n+1/2} halo (27 % of the
// tile against 16 %).
template <typename T>
struct Geo {
    static constexpr int FX = sizeof(T) == 4 ? 128 : 64, FY = 8, FT = FX * FY;
    static constexpr int EX = FX + 3, EY = FY + 3, ECELLS = EX * EY;   // E tile: x, y in [-1, +2]
    static constexpr int BX = FX + 2, BY = FY + 2, BCELLS = BX * BY;   // B^{n+1/2} tile: x, y in [-1, +1]
    static constexpr int EPER = (ECELLS + FT - 1) / FT;
    static constexpr int BPER = (BCELLS + FT - 1) / FT;
    // planes in flight per thread: FP32 two (1.87 against 1.98 ms; 128
    // VGPRs, a few bytes spilled at p >= 1), FP64 one (two measured slower:
    // 5.7 against 4.9 ms)
    static constexpr int PF = sizeof(T) == 4 ? 2 : 1;
};

template <typename T, int P>
struct JTile {
    static constexpr int FX = Geo<T>::FX, FY = Geo<T>::FY, FT = Geo<T>::FT;
    static constexpr int JX = FX + 2 * P, JY = FY + 2 * P, CELLS = JX * JY;
    static constexpr int PER = (CELLS + FT - 1) / FT;     // raw current cells per thread
    static constexpr int XITEMS = FX * JY;                // x-filtered cells per component
    static constexpr int XPER = (XITEMS + FT - 1) / FT;
};

__device__ __forceinline__ int wrapm(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

// alpha along an axis in "1 + small" form: f + (f- + f+ - 2 f)/6
template <typename T>
__device__ __forceinline__ T avg3(T fm, T f0, T fp, int lumped)
{
    return lumped ? f0 : f0 + (fm + fp - T(2) * f0) * T(1.0 / 6.0);
}

// one three-tap binomial pass (1,2,1)/4
template <typename T>
__device__ __forceinline__ T binom(T a, T b, T c)
{
    return T(0.25) * a + T(0.5) * b + T(0.25) * c;
}

// p cascaded three-tap passes over 2p+1 consecutive values v[0..2p]: the
// filtered value at the centre
template <typename T, int P>
__device__ __forceinline__ T binom_cascade(T (&v)[2 * P + 1])
{
    T w[2 * P + 1];
    for (int i = 0; i <= 2 * P; i++) w[i] = v[i];
    for (int r = 1; r <= P; r++)
        for (int i = 0; i + 2 * r <= 2 * P; i++) w[i] = binom(w[i], w[i + 1], w[i + 2]);
    return w[0];
}

template <typename T, int P>
__global__ __launch_bounds__(Geo<T>::FT) void k3_front(Coef<T> c, FrontArgs<T> a, const T *Bx_in, const T *By_in,
                                                       const T *Bz_in, int Lz)
{
    using G = Geo<T>;
    constexpr int FX = G::FX, FY = G::FY, FT = G::FT, EX = G::EX, EY = G::EY, ECELLS = G::ECELLS;
    constexpr int BX = G::BX, BY = G::BY, BCELLS = G::BCELLS, EPER = G::EPER, BPER = G::BPER;
    using JT = JTile<T, P>;
    __shared__ T sE[2][3][EY][EX];
    __shared__ T sB[3][3][BY][BX];
    __shared__ T sJ[3][JT::JY][JT::JX];
    __shared__ T sJx[3][JT::JY][FX];
    __shared__ double sred[FT / 64];

    const int nx = c.nx, ny = c.ny, nz = c.nz;
    const int tid = threadIdx.x, tx = tid % FX, ty = tid / FX;
    const int nwg = gridDim.x * gridDim.y * gridDim.z;
    const int lin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const int t_ = xcd_map(lin, nwg);
    const int gxy = gridDim.x * gridDim.y;
    const int X0 = (t_ % gridDim.x) * FX, Y0 = ((t_ % gxy) / gridDim.x) * FY;
    const int Z0 = (t_ / gxy) * Lz, Z1 = min(nz, Z0 + Lz);
    const size_t plane = (size_t)nx * ny;
    const bool has_j = a.J0[0] != nullptr;
    const T *Bin[3] = {Bx_in, By_in, Bz_in};

    // tile cells of this thread, fixed for the whole march
    unsigned eoff[EPER];
    int eidx[EPER];
    for (int u = 0; u < EPER; u++) {
        const int idx = tid + u * FT;
        eidx[u] = idx < ECELLS ? idx : -1;
        const int ix = idx % EX, iy = idx / EX;
        eoff[u] = (unsigned)wrapm(Y0 - 1 + iy, ny) * (unsigned)nx + wrapm(X0 - 1 + ix, nx);
    }
    unsigned boff[BPER];
    int bidx[BPER];
    bool bown[BPER];
    for (int u = 0; u < BPER; u++) {
        const int idx = tid + u * FT;
        bidx[u] = idx < BCELLS ? idx : -1;
        const int ix = idx % BX, iy = idx / BX;
        const int gx = X0 - 1 + ix, gy = Y0 - 1 + iy;
        boff[u] = (unsigned)wrapm(gy, ny) * (unsigned)nx + wrapm(gx, nx);
        bown[u] = bidx[u] >= 0 && ix >= 1 && ix <= FX && iy >= 1 && iy <= FY && gx < nx && gy < ny;
    }
    unsigned joff[JT::PER];
    int jidx[JT::PER];
    for (int u = 0; u < JT::PER; u++) {
        const int idx = tid + u * FT;
        jidx[u] = (has_j && idx < JT::CELLS) ? idx : -1;
        const int ix = idx % JT::JX, iy = idx / JT::JX;
        joff[u] = (unsigned)wrapm(Y0 - P + iy, ny) * (unsigned)nx + wrapm(X0 - P + ix, nx);
    }
    const bool out = X0 + tx < nx && Y0 + ty < ny;
    const unsigned own = out ? (unsigned)(Y0 + ty) * (unsigned)nx + (unsigned)(X0 + tx) : 0u;

    // prefetched planes (registers): a ring of PF sets, set (t - t0) % PF
    // holds what march step t stages
    constexpr int PF = G::PF;
    T eP[PF][EPER][3], bP[PF][BPER][3], jP[PF][JT::PER][3];
    auto fetchE = [&](int k, auto st) {
        constexpr int S = decltype(st)::value;
        const size_t zo = (size_t)wrapm(k, nz) * plane;
        for (int u = 0; u < EPER; u++)
            if (eidx[u] >= 0)
                for (int q = 0; q < 3; q++) eP[S][u][q] = a.E[q][zo + eoff[u]];
    };
    auto fetchB = [&](int k, auto st) {
        constexpr int S = decltype(st)::value;
        const size_t zo = (size_t)wrapm(k, nz) * plane;
        for (int u = 0; u < BPER; u++)
            if (bidx[u] >= 0)
                for (int q = 0; q < 3; q++) bP[S][u][q] = Bin[q][zo + boff[u]];
    };
    auto fetchJ = [&](int k, auto st) {
        constexpr int S = decltype(st)::value;
        const size_t zo = (size_t)wrapm(k, nz) * plane;
        for (int u = 0; u < JT::PER; u++)
            if (jidx[u] >= 0)
                for (int q = 0; q < 3; q++) jP[S][u][q] = a.J0[q][zo + joff[u]];
    };
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, PF - 1>;

    // z filter of the own column: level r keeps its two previous inputs
    T zin[P > 0 ? P : 1][2][3];
    for (int r = 0; r < (P > 0 ? P : 1); r++)
        for (int s = 0; s < 2; s++)
            for (int q = 0; q < 3; q++) zin[r][s][q] = T(0);

    // march steps t0 .. Z1 + 1: E plane t, B^{n+1/2} plane t - 1, current
    // plane t - 2 + P raw (t - 2 filtered), dE' plane t - 2.  Starting at
    // t0 fills the z filter (2P steps) and the B^{n+1/2} planes below Z0.
    const int t0 = min(Z0 - 1, Z0 + 2 - 2 * P);
    double acc = 0.0;
    fetchE(t0, S0{});
    fetchB(t0 - 1, S0{});
    if (has_j) fetchJ(t0 - 2 + P, S0{});
    if constexpr (PF == 2) {
        fetchE(t0 + 1, S1{});
        fetchB(t0, S1{});
        if (has_j) fetchJ(t0 - 1 + P, S1{});
    }
    auto body = [&](const int t, auto st) {
        constexpr int S = decltype(st)::value;
        const int se = (t - t0) & 1, sep = se ^ 1;          // E slots of planes t and t - 1
        // --- stage plane t of E and the raw current plane t - 2 + P
        for (int u = 0; u < EPER; u++)
            if (eidx[u] >= 0)
                for (int q = 0; q < 3; q++) (&sE[se][q][0][0])[eidx[u]] = eP[S][u][q];
        for (int u = 0; u < JT::PER; u++)
            if (jidx[u] >= 0)
                for (int q = 0; q < 3; q++) (&sJ[q][0][0])[jidx[u]] = jP[S][u][q];
        // B^{n-1/2} of plane t - 1: with one set in flight copied out so the
        // next plane can be fetched at once, with two read in place and
        // refilled after its last use
        T bold[PF == 1 ? BPER : 1][3];
        if constexpr (PF == 1)
            for (int u = 0; u < BPER; u++)
                for (int q = 0; q < 3; q++) bold[u][q] = bP[S][u][q];
        auto bget = [&](int u, int q) -> T {
            if constexpr (PF == 1) return bold[u][q];
            else return bP[S][u][q];
        };
        __syncthreads();
        // the planes of march step t + PF into the set just staged
        if (t + PF <= Z1 + 1) {
            fetchE(t + PF, st);
            if (has_j) fetchJ(t - 2 + P + PF, st);
        }
        if constexpr (PF == 1) fetchB(t, st);
        // --- B^{n+1/2} at plane t - 1 on the tile and its one-cell halo
        const int kb = t - 1;
        const int sb = (kb - t0 + 3) % 3;
        if (t > t0) {
            for (int u = 0; u < BPER; u++) {
                if (bidx[u] < 0) continue;
                const int ix = bidx[u] % BX, iy = bidx[u] / BX;   // E tile (ix, iy) is the same cell
                auto E0 = [&](int q, int dx, int dy) { return sE[sep][q][iy + dy][ix + dx]; };
                auto E1 = [&](int q) { return sE[se][q][iy][ix]; };   // plane kb + 1
                const T ex = E0(0, 0, 0), ey = E0(1, 0, 0), ez = E0(2, 0, 0);
                const T bx = bget(u, 0) - (c.tdy * (E0(2, 0, 1) - ez) - c.tdz * (E1(1) - ey));
                const T by = bget(u, 1) - (c.tdz * (E1(0) - ex) - c.tdx * (E0(2, 1, 0) - ez));
                const T bz = bget(u, 2) - (c.tdx * (E0(1, 1, 0) - ey) - c.tdy * (E0(0, 0, 1) - ex));
                sB[sb][0][iy][ix] = bx;
                sB[sb][1][iy][ix] = by;
                sB[sb][2][iy][ix] = bz;
                if (bown[u] && kb >= Z0 && kb < Z1) {
                    const size_t o = (size_t)kb * plane + boff[u];
                    a.B[0][o] = bx;
                    a.B[1][o] = by;
                    a.B[2][o] = bz;
                }
            }
        }
        if constexpr (PF == 2) fetchB(t + 1, st);
        // --- x filter of the staged current plane
        if (has_j) {
            for (int u = 0; u < JT::XPER; u++) {
                const int idx = tid + u * FT;
                if (idx >= JT::XITEMS) continue;
                const int x = idx % FX, y = idx / FX;
                for (int q = 0; q < 3; q++) {
                    T v[2 * P + 1];
                    for (int i = 0; i <= 2 * P; i++) v[i] = sJ[q][y][x + i];
                    sJx[q][y][x] = binom_cascade<T, P>(v);
                }
            }
        }
        __syncthreads();
        // --- y filter, then the z filter: the filtered current at plane t - 2
        T jf[3] = {T(0), T(0), T(0)};
        if (has_j) {
            T j2[3];
            for (int q = 0; q < 3; q++) {
                T v[2 * P + 1];
                for (int i = 0; i <= 2 * P; i++) v[i] = sJx[q][ty + i][tx];
                j2[q] = binom_cascade<T, P>(v);
            }
            if constexpr (P == 0) {
                for (int q = 0; q < 3; q++) jf[q] = j2[q];
            } else {
                for (int q = 0; q < 3; q++) {
                    T in = j2[q];
                    for (int r = 0; r < P; r++) {
                        const T o = binom(zin[r][0][q], zin[r][1][q], in);
                        zin[r][0][q] = zin[r][1][q];
                        zin[r][1][q] = in;
                        in = o;
                    }
                    jf[q] = in;
                }
            }
        }
        // --- dE' at plane t - 2 (own cell; B^{n+1/2} planes t - 3 .. t - 1)
        const int kd = t - 2;
        if (out && kd >= Z0 && kd < Z1) {
            const int s0 = (kd - t0 + 3) % 3, sm = (kd - 1 - t0 + 3) % 3, sp = (kd + 1 - t0 + 3) % 3;
            const int L = c.lumped;
            const int cx = tx + 1, cy = ty + 1;
            auto slot = [&](int dk) { return dk < 0 ? sm : (dk > 0 ? sp : s0); };
            auto azBz = [&](int di, int dj) {
                return avg3(sB[sm][2][cy + dj][cx + di], sB[s0][2][cy + dj][cx + di], sB[sp][2][cy + dj][cx + di], L);
            };
            auto ayBy = [&](int di, int dk) {
                const int s = slot(dk);
                return avg3(sB[s][1][cy - 1][cx + di], sB[s][1][cy][cx + di], sB[s][1][cy + 1][cx + di], L);
            };
            auto axBx = [&](int dj, int dk) {
                const int s = slot(dk);
                return avg3(sB[s][0][cy + dj][cx - 1], sB[s][0][cy + dj][cx], sB[s][0][cy + dj][cx + 1], L);
            };
            const T azbz = azBz(0, 0), ayby = ayBy(0, 0), axbx = axBx(0, 0);
            const T vx = c.tdy * (azbz - azBz(0, -1)) - c.tdz * (ayby - ayBy(0, -1)) - a.env_src * jf[0];
            const T vy = c.tdz * (axbx - axBx(0, -1)) - c.tdx * (azbz - azBz(-1, 0)) - a.env_src * jf[1];
            const T vz = c.tdx * (ayby - ayBy(-1, 0)) - c.tdy * (axbx - axBx(-1, 0)) - a.env_src * jf[2];
            const size_t o = (size_t)kd * plane + own;
            a.dEp[0][o] = vx;
            a.dEp[1][o] = vy;
            a.dEp[2][o] = vz;
            acc += (double)vx * vx + (double)vy * vy + (double)vz * vz;
        }
    };
    int t = t0;
    if constexpr (PF == 2)
        for (; t + 1 <= Z1 + 1; t += 2) {
            body(t, S0{});
            body(t + 1, S1{});
        }
    for (; t <= Z1 + 1; t++) body(t, S0{});
    if (a.partial != nullptr) {
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        const int lane = tid & 63, w = tid >> 6;
        __syncthreads();
        if (lane == 0) sred[w] = acc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int q = 0; q < FT / 64; q++) s += sred[q];
            a.partial[2 * lin] = s;
            a.partial[2 * lin + 1] = 0.0;
        }
    }
}

}  // namespace

int front3d_max_passes() { return 2; }

template <typename T>
hipError_t launch_front3d(const Coef<T> &c, int filter_passes, const FrontArgs<T> &a, const T *const Bin[3],
                          hipStream_t s, int *nwg)
{
    if (filter_passes < 0 || filter_passes > 2) return hipErrorInvalidValue;
    const int p = a.J0[0] ? filter_passes : 0;
    using G = Geo<T>;
    const void *k = p == 0 ? (const void *)k3_front<T, 0> : p == 1 ? (const void *)k3_front<T, 1>
                                                                   : (const void *)k3_front<T, 2>;
    // z chunks: one round of the resident workgroups, each chunk at least 16 planes
    static std::atomic<int> resident[3][MX_MAX_DEVICES];
    const int slots = per_device(resident[p], [k] {
        int o = 0, dev = 0, cu = 0;
        (void)hipGetDevice(&dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k, G::FT, 0) != hipSuccess || o < 1) o = 1;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu < 1) cu = 256;
        return o * cu;
    });
    const int gx = (c.nx + G::FX - 1) / G::FX, gy = (c.ny + G::FY - 1) / G::FY;
    int nzc = std::max(1, std::min(c.nz / 16, (slots + gx * gy - 1) / (gx * gy)));
    const int Lz = (c.nz + nzc - 1) / nzc;
    nzc = (c.nz + Lz - 1) / Lz;
    dim3 g(gx, gy, nzc);
    *nwg = g.x * g.y * g.z;
    if (p == 0) hipLaunchKernelGGL((k3_front<T, 0>), g, dim3(G::FT), 0, s, c, a, Bin[0], Bin[1], Bin[2], Lz);
    else if (p == 1) hipLaunchKernelGGL((k3_front<T, 1>), g, dim3(G::FT), 0, s, c, a, Bin[0], Bin[1], Bin[2], Lz);
    else hipLaunchKernelGGL((k3_front<T, 2>), g, dim3(G::FT), 0, s, c, a, Bin[0], Bin[1], Bin[2], Lz);
    return hipGetLastError();
}

template hipError_t launch_front3d<float>(const Coef<float> &, int, const FrontArgs<float> &, const float *const[3],
                                          hipStream_t, int *);
template hipError_t launch_front3d<double>(const Coef<double> &, int, const FrontArgs<double> &,
                                           const double *const[3], hipStream_t, int *);

}  // namespace mx
