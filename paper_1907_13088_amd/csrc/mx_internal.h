// Internal declarations shared by the host library and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "../../include/mx.h"

namespace mx {

// A launch-shape figure of the current device (resident workgroups of a
// kernel), computed on first use on each device and kept.  Host threads may
// race on the first use: each then computes the same value.
constexpr int MX_MAX_DEVICES = 64;
template <typename F>
inline int per_device(std::atomic<int> (&cache)[MX_MAX_DEVICES], F &&compute)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MX_MAX_DEVICES) return compute();
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        v = compute() + 1;   // stored biased by one: zero means "not yet computed"
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return v - 1;
}

// Per-grid scalar coefficients, computed on the host in FP64 and rounded
// once to the kernel type.  r_i = (c dt / d_i)^2, r_ij = (c dt)^2/(d_i d_j).
template <typename T>
struct Coef {
    int nx, ny, nz;
    T tdx, tdy, tdz;            // dt / d_i (curl prefactors)
    T src;                      // 4 pi dt (current prefactor)
    // 2D A (eqs matrixA_*_2d): TE  x+ = b + cxx Dyy x + cxy DxDy y
    //                                y+ = b + cyy Dxx y + cxy DxDy x
    //                          TM  z+ = b + czx Dxx z + czy Dyy z + czz DxxDyy z
    // 3D A (eqs matrixA_*): diagonal blocks a[i][0..2] = ((r_j-1)/6, (r_k-1)/6,
    // (r_j+r_k-1)/36) for the (j, k) axes cyclic after i; off-diagonal
    // o[i][j] = -r_ij / 6 multiplying Dbar_i Dbar_j alpha_k.
    T cxx, cyy, cxy, czx, czy, czz;
    T a3[3][3];
    T o3[3];                    // o3[0] = -r_yz/6 (yz pair), o3[1] = -r_zx/6, o3[2] = -r_xy/6
    int lumped;
};

// Sweep pass flags (runtime, uniform per launch)
enum : int {
    SW_FIRST = 1,     // iterate input is dE' itself (x_0 = dE')
    SW_LAST = 2,      // add the final iterate (or sum) to E
    SW_RESID = 4,     // accumulate FP64 norm of the last sweep's step
    SW_STORE = 8,     // store the final iterate (and sum) for a later pass
};

template <typename T>
struct SweepArgs {
    const T *x_in[3];     // iterate (standard) or delta (delta form), with halo
    const T *rhs[3];      // dE' (standard form)
    const T *s_in[3];     // running sum (delta form), increment (Chebyshev)
    T *x_out[3];
    T *s_out[3];
    T *E[3];
    double *partial;      // per-workgroup partial sums [nblocks][2] (TE, TM)
    // tolerance solve: the pass does nothing when *skip is set (its block
    // has met the stop test on the device); null: always run
    const int *skip;
    // Chebyshev form: per block (TE, TM) and sweep level of the pass, the
    // factors of the previous increment and of the residual
    T cheb[2][2][16];
};

// Device-side state of a tolerance solve within one step, per block (2D:
// TE, TM; 3D: block 0).  Passes of a block are queued ahead of the stop
// test; each pass's norm is reduced and tested on the device, which sets
// skip[b] once the block has converged (or has no work, or a norm is not
// finite), so the passes queued after it do nothing.
struct TolState {
    double rhsn[2];       // ||dE'|| per block
    double resid[2];      // ||x_(j+1) - x_j|| of the last pass run
    int skip[2];          // 1: further passes of the block do nothing
    int done[2];          // sweeps run
    int conv[2];          // met resid <= tol * rhsn
    int last[2];          // iterate buffer the last pass run wrote (-1: none)
    int nonfinite;        // bit 0: ||dE'||, bit 1: a residual
    int pad;
};

// Iterate forms of the 2D streaming sweep pass (compile time)
enum : int {
    FM_STD = 0,     // x_(j+1) = b + A x_j (Alg 1)
    FM_DELTA = 1,   // d_(j+1) = A d_j, s_(j+1) = s_j + d_(j+1)
    FM_CHEB = 2,    // Chebyshev semi-iteration on (1 - A) x = b
};

template <typename T>
struct FrontArgs {
    const T *E[3];
    T *B[3];
    const T *J0[3];       // may be null
    T env_src;            // env * 4 pi dt
    T *dEp[3];
    double *partial;      // per-workgroup ||dE'||^2 partials [nblocks][2], or null
};

// Workgroup barrier that orders LDS only: the streaming kernels exchange rows
// through LDS, never through global memory, so outstanding global loads (row
// prefetches) and stores may stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Work item of workgroup b (linear index) in a launch of n workgroups, such
// that each XCD receives one contiguous range of items.  Workgroups are dealt
// round-robin over the 8 XCDs (workgroup b runs on XCD b % 8), so XCD x holds
// q + (x < r) of them for n = 8 q + r; the map is a bijection of [0, n) for
// any n.  The kernels number their tiles x-fastest, so tiles that neighbour
// each other run on one XCD at the same time and share the L2 lines of their
// halos.
__device__ __forceinline__ int xcd_map(int b, int n)
{
    const int x = b & 7, j = b >> 3;
    const int q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + j;
}

// Element access by a 32-bit byte offset from a uniform base: lets the
// compiler use the scalar-base + vector-offset addressing form, one offset
// register shared by every component of a row.  Arrays are below 4 GiB.
// The access goes through a global-address-space pointer: field arrays are
// in device global memory, and a base pointer read from memory (a batch's
// grid descriptor) would otherwise be a generic pointer to the compiler,
// accessed by flat loads and stores with per-lane 64-bit addresses.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ T ld_off(const T *base, unsigned byte_off)
{
    return *(gptr<const T>)(reinterpret_cast<const char *>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ void st_off(T *base, unsigned byte_off, T v)
{
    *(gptr<T>)(reinterpret_cast<char *>(base) + byte_off) = v;
}

// Store that is not kept in the caches (non-temporal): for results that no
// kernel reads again soon, such as E at the end of a step
template <typename T>
__device__ __forceinline__ void st_off_nt(T *base, unsigned byte_off, T v)
{
    __builtin_nontemporal_store(v, (gptr<T>)(reinterpret_cast<char *>(base) + byte_off));
}

// One grid of a batch (device-resident descriptor)
template <typename T>
struct GridDesc {
    Coef<T> c;
    T *E[3];
    T *B[2][3];       // [0] the caller's buffers, [1] workspace (B ping-pongs per step)
    T *dEp[3];
    T *X[2][3];
    int nsx_f, nsx_s; // strips of the front and of the sweep pass
};

// Strip geometry of the row-streaming kernels.  An aligned strip writes a
// 128-byte aligned run of RX - 32 columns (16 halo columns on each side), so
// no cache line is written partly by two workgroups (on different XCDs);
// this pays where a kernel is bound by HBM traffic: the front pass, and
// sweep passes of at most 4 sweeps.  Deeper sweep passes are bound by
// issue, and keep the narrowest halo (k columns on each side).
constexpr bool front_aligned() { return true; }
constexpr bool stream_aligned(int k) { return k <= 4; }
constexpr int stream_halo(int k) { return stream_aligned(k) ? 16 : k; }
template <int RX>
constexpr int stream_width(int k) { return stream_aligned(k) ? RX - 32 : RX - 2 * k; }

namespace batch2d {
constexpr int STRIP = 256;                                    // threads (columns) per strip
inline int front_width() { return STRIP - 32; }   // aligned front strips
inline int sweep_width(int k) { return stream_width<STRIP>(k); }
template <typename T>
hipError_t launch_front(const GridDesc<T> *d, int ng, const int *items, int nitems, int L, int bin, hipStream_t s);
// the front and the first pass of k sweeps (3..6, FP32) in one launch over
// the front's items; writes iterate buffer 0
template <typename T>
hipError_t launch_front_sweep(const GridDesc<T> *d, int ng, const int *items, int nitems, int L, int k, int bin,
                              hipStream_t s);
constexpr int FUSE_KMIN = 3, FUSE_KMAX = 6;   // fused first-pass depths (FP32)
template <typename T>
hipError_t launch_sweep(const GridDesc<T> *d, int ng, const int *items, int nitems, int L, int k, bool first,
                        bool last, int xin, int xout, hipStream_t s);
constexpr int KMAX = 7;          // deepest batched pass (grouped or persistent)
// co-resident workgroups of the persistent kernel whose deepest pass has q
// sweeps (0: unsupported q)
template <typename T>
int persistent_blocks(int q);
// all nsteps steps in one cooperative launch: per step the front, then npass
// passes, the first nlow of q - 1 sweeps and the rest of q (fuse: the front
// and the first pass as one phase; FP32, first pass 3..6 deep).  No
// grid-wide barrier: each item waits for the previous phase of its own grid
// only.  cnt[0 .. ndone] (the claim counter, then ndone = ng * phases per
// step per-grid counters) is zeroed by the launch; *err must be zero at
// launch.
template <typename T>
hipError_t launch_persistent(const GridDesc<T> *d, int ng, const int *items_f, const int *items_s, int Lf, int Ls,
                             int nsteps, int q, int npass, int nlow, int bin0, unsigned *cnt, int ndone, int *err,
                             int fuse, hipStream_t s);
}  // namespace batch2d

// 2D launchers (k2d.hip)
template <typename T>
hipError_t launch_front_stream2d(const Coef<T> &c, int blocks, int filter_passes, const FrontArgs<T> &a,
                                 const T *const Bin[3], hipStream_t s, int *nwg);
template <typename T>
hipError_t launch_sweep2d(const Coef<T> &c, int blocks, int k, bool delta, int flags,
                          const SweepArgs<T> &a, hipStream_t s, int *nwg);
// one pass of k sweeps over a block set (1 TE, 2 TM, 3 both) with the
// row-streaming kernel; k in [1, stream2d_kmax(...)]
template <typename T>
hipError_t launch_stream2d(const Coef<T> &c, int block, int k, int form, int flags, const SweepArgs<T> &a,
                           hipStream_t s, int *nwg, int slots);
int stream2d_kmax(bool f64, int block, int form);
// the front and the first pass of k sweeps of both blocks (standard form,
// storing the iterate) in one row-streaming pass (k2fs.hip); available for
// the (dtype, k, filter passes) where front_sweep2d_ok holds
bool front_sweep2d_ok(bool f64, int k, int filter_passes);
template <typename T>
hipError_t launch_front_sweep2d(const Coef<T> &c, int filter_passes, int k, const FrontArgs<T> &fa,
                                const T *const Bin[3], const SweepArgs<T> &sa, hipStream_t s, int *nwg);
template <typename T>
hipError_t launch_update(int64_t n, int comp_mask, T *const E[3], const T *const X[3], hipStream_t s);

// mx_step on the scratch `ws` (ws_bytes) of device `device`, which is
// current: the body of mx_step_static (mx_api.cpp)
int step_on_scratch(const mx_config *cfg, void *stream, int device, void *ws, size_t ws_bytes, void *const E[3],
                    void *const B[3], void *const J0[3], int nsteps, const double *env, const int *replay,
                    mx_step_stats *stats);

// Single-launch tolerance solve of small 2D grids (k2small_impl.h): all
// passes of up to SMALL_MAX_STEPS steps in one cooperative launch, the stop
// test on the device, one read-back of the per-step records per launch.
constexpr int SMALL_MAX_STEPS = 64;
struct SmallStat {
    int done[2];          // sweeps per block (TE, TM)
    int conv[2];          // met the tolerance
    double resid[2];      // last step norm per block
    double rhsn[2];       // ||dE'|| per block
    int nonfinite;        // bit 0: ||dE'||, bit 1: a residual
    int pad;
};
template <typename T>
struct SmallArgs {
    Coef<T> c;
    T *E[3];
    T *B[2][3];           // step s reads B[s & 1][q], writes B[(s + 1) & 1][q] (active blocks)
    const T *J0[3];       // null: no current
    T *dEp[3];
    T *X[2][3];
    T *S[3];              // running sum (delta form)
    double *partial;      // per-workgroup FP64 partial norms [workgroups][2]
    unsigned *bar;        // grid barrier counters, zero at launch
    int *err;             // barrier time-out flag, zero at launch
    SmallStat *stat;      // [nsteps]
    const T *env_src;     // [nsteps] env * 4 pi dt of each step (device)
    double tol;
    int nsteps, blocks, spp, mmax, filter_passes;
    int ntx, nty;         // tiles per axis
};
// tiles of the grid (workgroups of the launch) and the co-resident limit of
// the kernel on the current device (0: no cooperative launch)
template <typename T>
void small_tiles(int nx, int ny, int *ntx, int *nty);
template <typename T>
int small_capacity(bool delta, int blocks);
template <typename T>
hipError_t launch_small(const SmallArgs<T> &a, bool delta, hipStream_t s);

// Particle push and charge-conserving deposition, 2D (kpic.hip)
template <typename T>
struct PicArgs {
    const T *E[3];        // E^n
    const T *B[3];        // B^{n-1/2}
    T *x, *y;             // positions (in: n, out: n + 1, wrapped into [0, L))
    T *ux, *uy, *uz;      // u = gamma v (in: n - 1/2, out: n + 1/2)
    T *J[3];              // J^{n+1/2} is added here
    int64_t np;
    int nx, ny;
    T dx, dy, dt;
    T th;                 // dt / 2: B^n = B^{n-1/2} - th curl E^n
    T h;                  // q dt / (2 m)
    T cx, cy, cz;         // -q w / (dy dt), -q w / (dx dt), q w / (dx dy)
    T Lx, Ly;             // nx dx, ny dy
};
template <typename T>
hipError_t launch_pic_push(const PicArgs<T> &a, bool zero_j, hipStream_t s);
template <typename T>
hipError_t launch_pic_charge(int64_t np, int nx, int ny, T dx, T dy, T cq, const T *x, const T *y, T *rho,
                             bool zero_rho, hipStream_t s);

// Fused 3D front (k3f.hip): Faraday into a.B from Bin, p <= front3d_max_passes()
// filter passes of the current, dE' (and its FP64 partial norms when
// a.partial is set); *nwg receives the workgroup count
int front3d_max_passes();
template <typename T>
hipError_t launch_front3d(const Coef<T> &c, int filter_passes, const FrontArgs<T> &a, const T *const Bin[3],
                          hipStream_t s, int *nwg);

// 3D launchers (k3d.hip)
template <typename T>
hipError_t launch_filter3d(const Coef<T> &c, int passes, const T *const J0[3], T *const Jf[3],
                           T *const tmp[3], hipStream_t s);
template <typename T>
hipError_t launch_faraday3d(const Coef<T> &c, const T *const E[3], T *const B[3], hipStream_t s);
template <typename T>
hipError_t launch_rhs3d(const Coef<T> &c, const T *const B[3], const T *const Jf[3], T env_src,
                        T *const dEp[3], double *partial, hipStream_t s, int *nwg);
// one pass of k sweeps over a 3D grid in iterate form `form`, k in
// [1, stream3d_kmax] (k3s.hip)
int stream3d_kmax(bool f64);
template <typename T>
hipError_t launch_stream3d(const Coef<T> &c, int k, int form, int flags, const SweepArgs<T> &a, hipStream_t s,
                           int *nwg);
template <typename T>
hipError_t launch_sweep3d(const Coef<T> &c, int k, int form, int flags, const SweepArgs<T> &a,
                          hipStream_t s, int *nwg);

// FP64 partial-sum reduction: out[0..1] = sum over nwg rows of partial[row][0..1]
hipError_t launch_reduce2(const double *partial, int nwg, double *out, hipStream_t s, const int *skip = nullptr);
// tolerance solve state: start a step from the reduced ||dE'||^2 per block
hipError_t launch_tol_init(TolState *st, const double *red, int nblk, hipStream_t s);
// after a pass of k sweeps of block b that wrote iterate buffer buf: the
// reduced step norm, the stop test against tol * ||dE'||
hipError_t launch_tol_decide(TolState *st, const double *red, int b, int k, int buf, double tol, hipStream_t s);

// Adjoint helpers (kadj.hip)
// Bbar += dt Lambda K v, and acc += sc v on the stepped components when acc
// is set
template <typename T>
hipError_t launch_adj_curlB(const Coef<T> &c, int ndim, int blocks, const T *const v[3],
                            T *const Bbar[3], T sc, T *const acc[3], hipStream_t s);
template <typename T>
hipError_t launch_adj_curlE(const Coef<T> &c, int ndim, int blocks, const T *const Bbar[3],
                            T *const Ebar[3], hipStream_t s);
template <typename T>
hipError_t launch_adj_source(const Coef<T> &c, int ndim, int passes, const T *const v[3],
                             T *const tmp1[3], T *const tmp2[3], T scale, T *const dJ0[3],
                             hipStream_t s);
template <typename T>
hipError_t launch_sources(int nx, int ny, int nsrc, int W, const int64_t *origins, const T *shapes,
                          const T *amps, T *const J0[3], T *const G[3], T *grad, bool project,
                          hipStream_t s);
template <typename T>
hipError_t launch_axpy3(int64_t n, int mask, bool zero, T a, const T *const x[3], T *const acc[3], hipStream_t s);

}  // namespace mx
