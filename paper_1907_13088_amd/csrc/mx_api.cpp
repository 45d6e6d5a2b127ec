// Host side of the C ABI declared in include/mx.h: validation, workspace
// layout, the per-step launch schedule (front pass, sweep passes, residual
// checks, E increment) and the transposed step.
#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "mx_internal.h"

using namespace mx;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(MX_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t ALIGN = 256;
size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

int64_t ncell_of(const mx_config *c) { return c->n[0] * c->n[1] * (c->ndim == 3 ? c->n[2] : 1); }
size_t elem_of(const mx_config *c) { return c->dtype == MX_F64 ? 8 : 4; }

// upper bound on workgroups of any launch that writes partial sums
int64_t max_wg(const mx_config *c)
{
    const int64_t nx = c->n[0], ny = c->n[1], nz = c->ndim == 3 ? c->n[2] : 1;
    // 2D front tiles 64x16, 2D sweep tiles 64x8 at the smallest, 3D 64x4 per plane
    const int64_t a = ((nx + 63) / 64) * ((ny + 3) / 4) * nz;
    // the streaming sweep launches at most one workgroup per (strip, row);
    // strips are at least 256 - 2 * 16 columns wide
    const int64_t b = ((nx + 223) / 224 + 1) * ny;
    return std::max(a, b);
}

// Sweeps per pass of each 2D block (TE, TM).  The LDS-tile kernel (variant
// 1) and the joint row-streaming kernel (variant 2) run both blocks in one
// pass; the per-block row-streaming kernels (variant 3) run each block on
// its own, as deep as its register windows allow.  Under a tolerance both
// blocks use the same depth, which is then also the granularity of the
// stopping test.
void pass_depths(const mx_config *c, int variant, int out[2])
{
    if (c->ndim == 3) {
        // 3D: z-marching passes of up to three sweeps (FP32; two in FP64),
        // as deep as allowed by default
        const int kmax = mx::stream3d_kmax(c->dtype == MX_F64);
        out[0] = out[1] = c->sweeps_per_pass > 0 ? std::min(c->sweeps_per_pass, kmax) : kmax;
        return;
    }
    const bool f64 = c->dtype == MX_F64;
    if (variant == 1) {
        // under a tolerance every pass ends in a host round trip for the
        // stop test: deeper passes make fewer of them
        const int k = c->sweeps_per_pass > 0 ? c->sweeps_per_pass : c->tol > 0.0 ? 8 : (f64 ? 4 : 5);
        out[0] = out[1] = k;
        return;
    }
    const bool tolmode = c->tol > 0.0;
    const bool delta = tolmode && c->form == MX_FORM_DELTA;
    const int form = c->solver == MX_SOLVER_CHEBYSHEV ? mx::FM_CHEB : delta ? mx::FM_DELTA : mx::FM_STD;
    const bool joint = (variant == 2 || variant == 4) && c->blocks == MX_ALL;
    const int kmax[2] = {mx::stream2d_kmax(f64, joint ? 3 : 1, form), mx::stream2d_kmax(f64, joint ? 3 : 2, form)};
    for (int b = 0; b < 2; b++) {
        int k = c->sweeps_per_pass > 0 ? c->sweeps_per_pass : kmax[b];
        if (tolmode && c->sweeps_per_pass <= 0) k = std::min(kmax[0], kmax[1]);
        out[b] = std::min(k, kmax[b]);
    }
}

// Workgroups of one row-streaming sweep pass on this grid, as the launcher
// cuts it (strips of stream_width(k) columns, chunks that fill two
// workgroups per CU but hold at least 4k rows).
int stream_workgroups(const mx_config *c, int variant, int ncu)
{
    int spp[2];
    pass_depths(c, variant, spp);
    const int k = std::max(spp[0], spp[1]);
    const long long nx = c->n[0], ny = c->n[1];
    const long long w = mx::stream_width<256>(k);
    const long long nsx = (nx + w - 1) / w;
    long long nsy = std::min(std::max(1LL, 2LL * ncu / nsx), ny);
    long long L = (ny + nsy - 1) / nsy;
    L = std::max(L, std::min(ny, 4LL * k));
    nsy = (ny + L - 1) / L;
    return (int)std::min(nsx * nsy, 0x7fffffffLL);
}

// workspace of the single-launch small-grid solve: per-step current
// factors and records, barrier counters and flag
size_t small_area()
{
    return up(SMALL_MAX_STEPS * sizeof(double)) + up(SMALL_MAX_STEPS * sizeof(SmallStat)) + up(4 * sizeof(unsigned));
}

// number of full-grid arrays in the workspace
int n_arrays(const mx_config *c)
{
    // dE' (3), two iterate buffers (6), running sum (3), a second B buffer
    // (3: the front writes B^{n+1/2} there, then the roles swap), then
    // 3D: filtered current and a filter temp (6; the separate filter passes
    // of p > 2 and the adjoint's current accumulator); the Chebyshev solve
    // adds a second increment buffer (3)
    if (c->ndim == 2) return c->solver == MX_SOLVER_CHEBYSHEV ? 18 : 15;
    return c->solver == MX_SOLVER_CHEBYSHEV ? 24 : 21;
}

}  // namespace

namespace mx {
// error reporting shared with the batch entry points
int api_fail(int code, const char *msg) { return fail(code, "%s", msg); }
}  // namespace mx

struct mx_grid {
    mx_config cfg;
    hipStream_t stream;
    int device;
    char *ws;
    size_t ws_bytes;
    int64_t ncell;
    int64_t step;
    void *E[3], *B[3], *J0[3];
    bool bound, has_j;
    void *dEp[3], *X[2][3], *S[3], *Bws[3], *Jf[3], *Jt[3];
    void *D2[3];          // Chebyshev solve: the increment buffer paired with S
    int bloc[3];          // 2D: where component q of B currently lives (0 user, 1 workspace)
    double *partial;      // device
    double *red;          // device, 2 doubles
    double *hred = nullptr;   // pinned host memory for read-backs (a TolState)
    TolState hbuf;            // pageable read-back target when hred is not set
    // single-launch small-grid solve: device areas in the workspace, and
    // pageable host copies (the per-step records and current factors)
    void *small_env;
    SmallStat *small_stat;
    unsigned *small_bar;      // [0..2] barrier, [3] time-out flag
    SmallStat hstat[SMALL_MAX_STEPS];
    double henv[SMALL_MAX_STEPS];
    TolState *tol;        // device: the tolerance solve's state within a step
    int spec[2] = {1, 1}; // passes per block the last tolerance solve ran (queued ahead next step)
    int spp[2];           // sweeps per pass of the TE and TM blocks (3D: [0])
    int variant;          // 2D sweep kernel in use: 1 LDS tile, 2 row streaming (blocks
                          // together), 3 row streaming (each block on its own), 4 as 2
                          // with the front fused into the first pass where possible
    Coef<float> cf;
    Coef<double> cd;
    // Chebyshev solve: per block, the factors (previous increment, residual)
    // of sweep k, for k < cfg.sweeps
    std::vector<double> cheb[2][2];
    // timing (mx_profile_*)
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<int> ev_cat;          // category per event pair
    int64_t launches[MX_PROF_NCAT] = {};
    double bytes[MX_PROF_NCAT] = {};
};

namespace {

// bracket one launch with events when profiling is on
struct ProfScope {
    mx_grid *g;
    int cat;
    hipEvent_t e1 = nullptr;
    ProfScope(mx_grid *g_, int cat_, double bytes) : g(g_), cat(cat_)
    {
        if (!g->prof) return;
        if (g->ev_used + 2 > g->ev_pool.size()) {
            for (int i = 0; i < 64; i++) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) { g->prof = false; return; }
                g->ev_pool.push_back(e);
            }
        }
        hipEvent_t e0 = g->ev_pool[g->ev_used];
        e1 = g->ev_pool[g->ev_used + 1];
        g->ev_used += 2;
        g->ev_cat.push_back(cat);
        (void)hipEventRecord(e0, g->stream);
        g->launches[cat] += 1;
        g->bytes[cat] += bytes;
    }
    ~ProfScope()
    {
        if (e1) (void)hipEventRecord(e1, g->stream);
    }
};

}  // namespace

// Chebyshev semi-iteration for (1 - A) x = b on a 2D block whose A has its
// spectrum in [0, rho]: 1 - A lies in [1 - rho, 1], with centre theta and
// half width delta, s1 = theta / delta.  Sweep k forms the residual
// r_k = b + A x_k - x_k, the increment d_k = f_k d_(k-1) + g_k r_k and
// x_(k+1) = x_k + d_k, where w_0 = 1/s1, f_0 = 0, g_0 = 1/theta and
// w_k = 1/(2 s1 - w_(k-1)), f_k = w_k w_(k-1), g_k = 2 w_k / delta (the
// three-term recurrence of the Chebyshev polynomials on that interval).
// rho is the top of the block symbol over the Brillouin zone: 2/3 for TE at
// any dt; for TM the largest corner value of the bilinear symbol
// (2/3)(1-rx) sx + (2/3)(1-ry) sy - (4/9)(1-rx-ry) sx sy, s_i in [0, 1].
static void fill_cheb(const mx_config *c, int n, std::vector<double> out[2][2])
{
    const double rx = c->dt * c->dt / (c->d[0] * c->d[0]), ry = c->dt * c->dt / (c->d[1] * c->d[1]);
    // 2D: TE 2/3, TM the largest corner of its bilinear symbol; 3D (cubic
    // cells, one block, index 0): 8/9 at any dt
    const double rho[2] = {c->ndim == 3 ? 8.0 / 9.0 : 2.0 / 3.0,
                           std::max({2.0 / 3.0 * (1.0 - rx), 2.0 / 3.0 * (1.0 - ry), 8.0 / 9.0 - 2.0 / 9.0 * (rx + ry)})};
    n = std::max(n, 1);
    for (int b = 0; b < 2; b++) {
        const double theta = 1.0 - rho[b] / 2.0, delta = rho[b] / 2.0, s1 = theta / delta;
        out[b][0].assign(n, 0.0);
        out[b][1].assign(n, 0.0);
        double wp = 0.0;
        for (int k = 0; k < n; k++) {
            if (k == 0) {
                wp = 1.0 / s1;
                out[b][0][0] = 0.0;
                out[b][1][0] = 1.0 / theta;
            } else {
                const double w = 1.0 / (2.0 * s1 - wp);
                out[b][0][k] = w * wp;
                out[b][1][k] = 2.0 * w / delta;
                wp = w;
            }
        }
    }
}

template <typename T>
static void fill_coef(const mx_config *c, Coef<T> &k)
{
    const double dt = c->dt;
    const double dx = c->d[0], dy = c->d[1], dz = c->ndim == 3 ? c->d[2] : 1.0;
    const double rx = dt * dt / (dx * dx), ry = dt * dt / (dy * dy), rz = dt * dt / (dz * dz);
    const double rxy = dt * dt / (dx * dy), ryz = dt * dt / (dy * dz), rzx = dt * dt / (dz * dx);
    k.nx = (int)c->n[0];
    k.ny = (int)c->n[1];
    k.nz = c->ndim == 3 ? (int)c->n[2] : 1;
    k.tdx = (T)(dt / dx);
    k.tdy = (T)(dt / dy);
    k.tdz = (T)(dt / dz);
    k.src = (T)(c->four_pi * dt);
    k.cxx = (T)((ry - 1.0) / 6.0);
    k.cyy = (T)((rx - 1.0) / 6.0);
    k.cxy = (T)(-rxy / 6.0);
    k.czx = (T)((rx - 1.0) / 6.0);
    k.czy = (T)((ry - 1.0) / 6.0);
    k.czz = (T)((rx + ry - 1.0) / 36.0);
    const double r[3] = {rx, ry, rz};
    for (int i = 0; i < 3; i++) {
        const int j = (i + 1) % 3, l = (i + 2) % 3;
        k.a3[i][0] = (T)((r[j] - 1.0) / 6.0);
        k.a3[i][1] = (T)((r[l] - 1.0) / 6.0);
        k.a3[i][2] = (T)((r[j] + r[l] - 1.0) / 36.0);
    }
    k.o3[0] = (T)(-ryz / 6.0);
    k.o3[1] = (T)(-rzx / 6.0);
    k.o3[2] = (T)(-rxy / 6.0);
    k.lumped = c->lumped;
}

// Lay a grid out on a validated config and a workspace of at least
// mx_workspace_size bytes: the sweep-kernel choice, the arrays of the
// workspace, the coefficients.  Allocates nothing (the caller sets hred, or
// leaves it null for pageable read-backs into hbuf).
static void grid_setup(mx_grid *g, const mx_config *cfg, hipStream_t stream, int device, char *ws, size_t ws_bytes)
{
    g->cfg = *cfg;
    g->stream = stream;
    g->device = device;
    g->ws = ws;
    g->ws_bytes = ws_bytes;
    g->ncell = ncell_of(cfg);
    g->step = 0;
    g->bound = false;
    g->has_j = false;
    g->hred = nullptr;
    // library choice: FP32 runs both blocks in one pass (7 sweeps deep),
    // the front fused with the first pass where a kernel exists for it
    // (4096^2, m = 20, p = 3: 0.648 against 0.702 ms per step); FP64, whose
    // joint passes are only 3 deep, runs each block on its own (TE 5, TM 8
    // deep), which moves fewer bytes per step; so does the Chebyshev solve
    // (joint passes 5 deep in FP32, per block 8 and 12: measured 0.46
    // against 0.60 ms per 4096^2 step at 7 sweeps).  A grid too small for
    // the row-streaming passes to occupy half the CUs runs the LDS-tile
    // kernel instead (128^2 to 768^2: 1.4 to 2.8 times faster per step; the
    // Chebyshev solve has no tile form)
    g->variant = cfg->variant > 0 ? cfg->variant
                                  : (cfg->dtype == MX_F64 || cfg->solver == MX_SOLVER_CHEBYSHEV ? 3 : 4);
    if (cfg->variant == 0 && cfg->ndim == 2 && cfg->solver != MX_SOLVER_CHEBYSHEV) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cu < 1)
            cu = 256;
        if (stream_workgroups(cfg, g->variant, cu) < cu / 2) g->variant = 1;
    }
    pass_depths(cfg, g->variant, g->spp);
    const size_t arr = up((size_t)g->ncell * elem_of(cfg));
    char *p = g->ws;
    auto take = [&](void **dst) { *dst = p; p += arr; };
    for (int q = 0; q < 3; q++) take(&g->dEp[q]);
    for (int b = 0; b < 2; b++)
        for (int q = 0; q < 3; q++) take(&g->X[b][q]);
    for (int q = 0; q < 3; q++) take(&g->S[q]);
    for (int q = 0; q < 3; q++) g->D2[q] = nullptr;
    if (cfg->ndim == 2) {
        for (int q = 0; q < 3; q++) take(&g->Bws[q]);
        for (int q = 0; q < 3; q++) g->Jf[q] = g->Jt[q] = nullptr;
        if (cfg->solver == MX_SOLVER_CHEBYSHEV)
            for (int q = 0; q < 3; q++) take(&g->D2[q]);
    } else {
        for (int q = 0; q < 3; q++) take(&g->Jf[q]);
        for (int q = 0; q < 3; q++) take(&g->Jt[q]);
        for (int q = 0; q < 3; q++) take(&g->Bws[q]);
        if (cfg->solver == MX_SOLVER_CHEBYSHEV)
            for (int q = 0; q < 3; q++) take(&g->D2[q]);
    }
    g->partial = (double *)p;
    p += up((size_t)max_wg(cfg) * 2 * sizeof(double));
    g->red = (double *)p;
    p += up(8 * sizeof(double));
    g->tol = (TolState *)p;
    p += up(sizeof(TolState));
    g->small_env = nullptr;
    g->small_stat = nullptr;
    g->small_bar = nullptr;
    if (cfg->ndim == 2) {
        g->small_env = p;
        p += up(SMALL_MAX_STEPS * sizeof(double));
        g->small_stat = (SmallStat *)p;
        p += up(SMALL_MAX_STEPS * sizeof(SmallStat));
        g->small_bar = (unsigned *)p;
    }
    for (int q = 0; q < 3; q++) { g->E[q] = g->B[q] = g->J0[q] = nullptr; g->bloc[q] = 0; }
    fill_coef(cfg, g->cf);
    fill_coef(cfg, g->cd);
    if (cfg->solver == MX_SOLVER_CHEBYSHEV) fill_cheb(cfg, cfg->sweeps, g->cheb);
}

extern "C" {

const char *mx_last_error(void) { return g_err.c_str(); }

int mx_config_default(mx_config *cfg)
{
    if (!cfg) return fail(MX_EINVAL, "cfg is NULL");
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->ndim = 2;
    cfg->n[0] = cfg->n[1] = cfg->n[2] = 1;
    cfg->d[0] = cfg->d[1] = cfg->d[2] = 1.0;
    cfg->dtype = MX_F32;
    cfg->blocks = MX_ALL;
    cfg->sweeps = 20;
    cfg->four_pi = 4.0 * M_PI;
    cfg->form = MX_FORM_STANDARD;
    return MX_OK;
}

int mx_validate(const mx_config *c, int *warn)
{
    if (warn) *warn = 0;
    if (!c) return fail(MX_EINVAL, "cfg is NULL");
    if (c->ndim != 2 && c->ndim != 3) return fail(MX_EINVAL, "ndim must be 2 or 3 (got %d)", c->ndim);
    for (int a = 0; a < c->ndim; a++) {
        if (c->n[a] < 1 || c->n[a] > (1LL << 30))
            return fail(MX_EINVAL, "n[%d] = %lld out of range [1, 2^30]", a, (long long)c->n[a]);
        if (!(c->d[a] > 0.0) || !std::isfinite(c->d[a]))
            return fail(MX_EINVAL, "d[%d] must be positive and finite", a);
    }
    if (ncell_of(c) > (1LL << 40)) return fail(MX_EINVAL, "too many cells");
    if (c->ndim == 2 && (double)ncell_of(c) * (c->dtype == MX_F64 ? 8 : 4) >= 4294967296.0)
        return fail(MX_EINVAL, "2D field arrays must be below 4 GiB (32-bit byte offsets)");
    if (c->ndim == 3 && (double)c->n[0] * (double)c->n[1] >= 4294967296.0)
        return fail(MX_EINVAL, "3D planes must hold fewer than 2^32 cells (32-bit in-plane offsets)");
    if (c->dtype != MX_F32 && c->dtype != MX_F64) return fail(MX_EINVAL, "dtype must be MX_F32 or MX_F64");
    if (c->ndim == 2 && (c->blocks < 1 || c->blocks > 3)) return fail(MX_EINVAL, "blocks must be MX_TE, MX_TM or MX_ALL");
    if (c->ndim == 3 && c->blocks != MX_ALL) return fail(MX_EINVAL, "3D grids step all components (MX_ALL)");
    if (c->sweeps < 0 || c->sweeps > 1000000) return fail(MX_EINVAL, "sweeps out of range");
    if (!(c->tol >= 0.0) || !std::isfinite(c->tol)) return fail(MX_EINVAL, "tol must be finite and >= 0");
    if (c->filter_passes < 0 || c->filter_passes > 4) return fail(MX_EINVAL, "filter_passes must be in [0, 4]");
    if (c->lumped != 0 && c->lumped != 1) return fail(MX_EINVAL, "lumped must be 0 or 1");
    if (!std::isfinite(c->four_pi)) return fail(MX_EINVAL, "four_pi must be finite");
    if (c->form != MX_FORM_STANDARD && c->form != MX_FORM_DELTA) return fail(MX_EINVAL, "bad form");
    if (c->solver != MX_SOLVER_ALG1 && c->solver != MX_SOLVER_CHEBYSHEV) return fail(MX_EINVAL, "bad solver");
    if (c->solver == MX_SOLVER_CHEBYSHEV) {
        if (c->ndim == 3 && !(c->d[0] == c->d[1] && c->d[1] == c->d[2]))
            return fail(MX_EINVAL, "the 3D Chebyshev solve is defined for cubic cells");
        if (c->variant == 1) return fail(MX_EINVAL, "the Chebyshev solve runs on the row-streaming kernels (variant 0, 2 or 3)");
        if (c->form != MX_FORM_STANDARD) return fail(MX_EINVAL, "the Chebyshev solve uses the standard form");
        if (c->lumped) return fail(MX_EINVAL, "the lumped scheme has A = 0: no solve to accelerate");
    }
    if (c->sweeps_per_pass < 0 || c->sweeps_per_pass > 16) return fail(MX_EINVAL, "sweeps_per_pass must be in [0, 16]");
    if (c->variant < 0 || c->variant > 4) return fail(MX_EINVAL, "variant must be 0, 1, 2, 3 or 4");
    if (c->variant == 1 && c->sweeps_per_pass > 8)
        return fail(MX_EINVAL, "the LDS-tile kernel runs at most 8 sweeps per pass");
    if (c->ndim == 3 && c->sweeps_per_pass > mx::stream3d_kmax(c->dtype == MX_F64))
        return fail(MX_EINVAL, "3D grids run at most three sweeps per pass in FP32, two in FP64");
    if (!(c->dt > 0.0) || !std::isfinite(c->dt)) return fail(MX_EINVAL, "dt must be positive and finite");
    double s = 0.0;
    for (int a = 0; a < c->ndim; a++) s += 1.0 / (c->d[a] * c->d[a]);
    const double dt_cfl = 1.0 / std::sqrt(s);
    if (c->dt > dt_cfl * (1.0 + 1e-12))
        return fail(MX_ECFL, "dt = %.17g exceeds the stability limit %.17g", c->dt, dt_cfl);
    if (c->ndim == 3) {
        const double dmin = std::min(c->d[0], std::min(c->d[1], c->d[2]));
        if (c->dt > dmin / std::sqrt(2.0) && warn) *warn |= MX_WARN_NOCONV_GUARANTEE;
    }
    return MX_OK;
}

int mx_workspace_size(const mx_config *c, size_t *bytes)
{
    int rc = mx_validate(c, nullptr);
    if (rc) return rc;
    if (!bytes) return fail(MX_EINVAL, "bytes is NULL");
    const size_t arr = up((size_t)ncell_of(c) * elem_of(c));
    *bytes = n_arrays(c) * arr + up((size_t)max_wg(c) * 2 * sizeof(double)) + up(8 * sizeof(double)) +
             up(sizeof(TolState)) + (c->ndim == 2 ? small_area() : 0);
    return MX_OK;
}

int mx_init(const mx_config *cfg, void *stream, void *workspace, size_t workspace_bytes, mx_grid **out)
{
    if (!out) return fail(MX_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = mx_validate(cfg, nullptr);
    if (rc) return rc;
    size_t need = 0;
    mx_workspace_size(cfg, &need);
    if (!workspace) return fail(MX_EWORKSPACE, "workspace is NULL (%zu bytes needed)", need);
    if (workspace_bytes < need)
        return fail(MX_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, need);
    if (((uintptr_t)workspace) % ALIGN) return fail(MX_EINVAL, "workspace must be %zu-byte aligned", ALIGN);
    hipPointerAttribute_t attr;
    HIPCHK(hipPointerGetAttributes(&attr, workspace));
    if (attr.type != hipMemoryTypeDevice) return fail(MX_EINVAL, "workspace is not device memory");
    HIPCHK(hipSetDevice(attr.device));

    mx_grid *g = new mx_grid();
    grid_setup(g, cfg, (hipStream_t)stream, attr.device, (char *)workspace, workspace_bytes);
    // pinned host memory: the tolerance solve reads its state back by DMA
    // rather than through a staged pageable copy
    const size_t hbytes = std::max(sizeof(TolState), SMALL_MAX_STEPS * (sizeof(SmallStat) + sizeof(double)));
    if (hipHostMalloc((void **)&g->hred, hbytes, hipHostMallocDefault) != hipSuccess) {
        delete g;
        return fail(MX_EDEVICE, "pinned host buffer of %zu bytes could not be allocated", hbytes);
    }
    *out = g;
    return MX_OK;
}

int mx_bind_fields(mx_grid *g, void *const E[3], void *const B[3])
{
    if (!g || !E || !B) return fail(MX_EINVAL, "NULL argument");
    for (int q = 0; q < 3; q++)
        if (!E[q] || !B[q]) return fail(MX_EINVAL, "field component %d is NULL", q);
    for (int q = 0; q < 3; q++) { g->E[q] = E[q]; g->B[q] = B[q]; g->bloc[q] = 0; }
    g->bound = true;
    return MX_OK;
}

int mx_set_current(mx_grid *g, void *const J0[3])
{
    if (!g) return fail(MX_EINVAL, "grid is NULL");
    if (!J0) { g->has_j = false; for (int q = 0; q < 3; q++) g->J0[q] = nullptr; return MX_OK; }
    for (int q = 0; q < 3; q++)
        if (!J0[q]) return fail(MX_EINVAL, "J0 component %d is NULL", q);
    for (int q = 0; q < 3; q++) g->J0[q] = J0[q];
    g->has_j = true;
    return MX_OK;
}

int mx_get_step(mx_grid *g, int64_t *n)
{
    if (!g || !n) return fail(MX_EINVAL, "NULL argument");
    *n = g->step;
    return MX_OK;
}

int mx_set_step(mx_grid *g, int64_t n)
{
    if (!g) return fail(MX_EINVAL, "NULL argument");
    g->step = n;
    return MX_OK;
}

int mx_get_sweeps_per_pass(mx_grid *g, int *k)
{
    if (!g || !k) return fail(MX_EINVAL, "NULL argument");
    const mx_config &c = g->cfg;
    *k = (c.ndim == 3 || (c.blocks & 1)) ? g->spp[0] : g->spp[1];
    return MX_OK;
}

int mx_get_block_sweeps_per_pass(mx_grid *g, int k[2])
{
    if (!g || !k) return fail(MX_EINVAL, "NULL argument");
    k[0] = g->spp[0];
    k[1] = g->spp[1];
    return MX_OK;
}

int mx_destroy(mx_grid *g)
{
    if (!g) return MX_OK;
    for (hipEvent_t e : g->ev_pool) (void)hipEventDestroy(e);
    if (g->hred) (void)hipHostFree(g->hred);
    delete g;
    return MX_OK;
}

int mx_profile_enable(mx_grid *g, int on)
{
    if (!g) return fail(MX_EINVAL, "grid is NULL");
    if (on < 0 || on > 2) return fail(MX_EINVAL, "on must be 0 (pause), 1 (reset and record) or 2 (resume)");
    g->prof = on != 0;
    if (on == 1) {
        g->ev_used = 0;
        g->ev_cat.clear();
        for (int i = 0; i < MX_PROF_NCAT; i++) { g->launches[i] = 0; g->bytes[i] = 0.0; }
    }
    return MX_OK;
}

int mx_profile_read(mx_grid *g, mx_profile *out)
{
    if (!g || !out) return fail(MX_EINVAL, "NULL argument");
    HIPCHK(hipSetDevice(g->device));
    HIPCHK(hipStreamSynchronize(g->stream));
    for (int i = 0; i < MX_PROF_NCAT; i++) { out->launches[i] = g->launches[i]; out->bytes[i] = g->bytes[i]; out->ms[i] = 0.0; }
    for (size_t p = 0; p < g->ev_cat.size(); p++) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, g->ev_pool[2 * p], g->ev_pool[2 * p + 1]));
        out->ms[g->ev_cat[p]] += ms;
    }
    return MX_OK;
}

}  // extern "C"

namespace {

template <typename T>
const Coef<T> &coef(const mx_grid *g);
template <>
const Coef<float> &coef<float>(const mx_grid *g) { return g->cf; }
template <>
const Coef<double> &coef<double>(const mx_grid *g) { return g->cd; }

int block_mask_comps(int ndim, int b) { return ndim == 3 ? 7 : (b == 0 ? 3 : 4); }

// Sweep arguments of one pass: input iterate buffer cb (-1: the right-hand
// side itself), output buffer ob; the Chebyshev increments ping-pong with
// the iterate (a pass reads its neighbours' halo increments, so none is
// updated in place; before the first sweep there is none: the kernel
// ignores the values it then reads, which hit the cache lines of dE').
template <typename T>
SweepArgs<T> pass_args(const mx_grid *g, void *const rhs[3], int cb, int ob, bool first, bool cheb,
                       void *const E_fuse[3])
{
    SweepArgs<T> a{};
    for (int q = 0; q < 3; q++) {
        a.rhs[q] = (const T *)rhs[q];
        a.x_in[q] = (const T *)(cb < 0 ? rhs[q] : g->X[cb][q]);
        a.s_in[q] = (const T *)g->S[q];
        a.x_out[q] = (T *)g->X[ob][q];
        a.s_out[q] = (T *)g->S[q];
        a.E[q] = E_fuse ? (T *)E_fuse[q] : nullptr;
    }
    a.partial = g->partial;
    a.skip = nullptr;
    if (cheb) {
        void *const *Din = cb == 1 ? g->D2 : g->S;
        void *const *Dout = ob == 1 ? g->D2 : g->S;
        for (int q = 0; q < 3; q++) {
            a.s_in[q] = (const T *)(first ? rhs[q] : Din[q]);
            a.s_out[q] = (T *)Dout[q];
        }
    }
    return a;
}

// Chebyshev factors of a pass of kk sweeps of block b whose first sweep is
// sweep number `done` of the solve (level l runs sweep done + l)
template <typename T>
void pass_cheb(const mx_grid *g, int b, int done, int kk, SweepArgs<T> &a)
{
    for (int l = 0; l < kk; l++) {
        const size_t ix = (size_t)(done + l);
        const bool ok = ix < g->cheb[b][0].size();
        a.cheb[b][0][l] = (T)(ok ? g->cheb[b][0][ix] : 0.0);
        a.cheb[b][1][l] = (T)(ok ? g->cheb[b][1][ix] : 0.0);
    }
}

// Arrays a pass touches per component (the algorithmic byte count of the
// profiler): the iterate (or dE' on the first pass) with halo, dE'
// (standard form), the running sum (delta form) or the increments
// (Chebyshev form), the stored iterate, or E read and written.
int pass_arrays(bool cheb, bool delta, bool first, bool last)
{
    if (cheb) return (first ? 1 : 3) + 2;
    if (!delta) return (first ? 1 : 2) + (last ? 2 : 1);
    return (first ? 1 : 2) + 2;
}

// Tolerance solve: Alg 1 (or the Chebyshev solve) with the stop test of
// each block.  Each block runs in passes of its own (2D: TE and TM; 3D: one
// block), of spp sweeps (the last one shorter where m_max ends the
// count).  Passes are queued ahead of the stop test: each is followed
// by the reduction of its step norm and the test on the device, which makes
// the passes queued after it do nothing once the block has converged.  The
// host reads the state back when the queued passes of every block have run:
// first as many per block as it ran at the previous step, then one more at
// a time.  The sweep counts and iterates equal those of testing after every
// pass on the host; the host waits about once per step instead of once per
// pass.
template <typename T>
int solve_tol(mx_grid *g, void *const rhs[3], const int *target_in, const T **res, mx_step_stats *st)
{
    const mx_config &c = g->cfg;
    const Coef<T> &k = coef<T>(g);
    const int nblk = c.ndim == 3 ? 1 : 2;
    const bool delta = c.form == MX_FORM_DELTA;
    const bool cheb = c.solver == MX_SOLVER_CHEBYSHEV;
    const int form = cheb ? FM_CHEB : delta ? FM_DELTA : FM_STD;
    bool active[2] = {false, false};
    int target[2] = {0, 0};
    for (int b = 0; b < nblk; b++) {
        active[b] = c.ndim == 3 || (c.blocks & (1 << b));
        target[b] = active[b] ? target_in[b] : 0;
    }
    if (cheb && (int)g->cheb[0][0].size() < std::max(target[0], target[1]))
        fill_cheb(&c, std::max(target[0], target[1]), g->cheb);
    TolState *hs = g->hred ? (TolState *)g->hred : &g->hbuf;
    bool have = false;
    auto read_back = [&]() -> int {
        HIPCHK(hipMemcpyAsync(hs, g->tol, sizeof(TolState), hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
        have = true;
        if (hs->nonfinite & 1)
            return fail(MX_ENONFINITE, "step %lld: norm of dE' is not finite", (long long)g->step);
        if (hs->nonfinite & 2)
            return fail(MX_ENONFINITE, "step %lld: a residual norm is not finite", (long long)g->step);
        return MX_OK;
    };
    int enq[2] = {0, 0}, swe[2] = {0, 0}, ahead[2];
    bool open[2];
    for (int b = 0; b < 2; b++) {
        ahead[b] = std::max(1, g->spec[b]);
        open[b] = b < nblk && target[b] > 0;
    }
    for (;;) {
        bool any = false;
        for (int b = 0; b < nblk; b++) {
            if (!open[b]) continue;
            any = true;
            const int spp = g->spp[b];
            const int *skip = &g->tol->skip[b];
            while (enq[b] < ahead[b] && swe[b] < target[b]) {
                const int kk = std::min(spp, target[b] - swe[b]);
                const bool first = enq[b] == 0;
                const int cb = first ? -1 : (enq[b] - 1) & 1, ob = enq[b] & 1;
                SweepArgs<T> a = pass_args<T>(g, rhs, cb, ob, first, cheb, nullptr);
                a.skip = skip;
                if (cheb) pass_cheb<T>(g, b, swe[b], kk, a);
                const int flags = (first ? SW_FIRST : 0) | SW_RESID | SW_STORE;
                int nwg = 0;
                hipError_t e;
                {
                    const int ncomp = c.ndim == 3 ? 3 : (b == 0 ? 2 : 1);
                    ProfScope ps(g, MX_PROF_SWEEP,
                                 (double)g->ncell * sizeof(T) * pass_arrays(cheb, delta, first, false) * ncomp);
                    if (c.ndim == 2 && g->variant == 1)
                        e = launch_sweep2d<T>(k, 1 << b, kk, delta, flags, a, g->stream, &nwg);
                    else if (c.ndim == 2)
                        e = launch_stream2d<T>(k, 1 << b, kk, form, flags, a, g->stream, &nwg, 0);
                    else
                        e = launch_sweep3d<T>(k, kk, form, flags, a, g->stream, &nwg);
                }
                if (e != hipSuccess) return fail(MX_EDEVICE, "sweep launch: %s", hipGetErrorString(e));
                {
                    ProfScope ps(g, MX_PROF_OTHER, 0.0);
                    HIPCHK(launch_reduce2(g->partial, nwg, g->red, g->stream, skip));
                    HIPCHK(launch_tol_decide(g->tol, g->red, b, kk, ob, c.tol, g->stream));
                }
                enq[b]++;
                swe[b] += kk;
            }
        }
        if (!any) break;
        const int rc = read_back();
        if (rc) return rc;
        for (int b = 0; b < nblk; b++) {
            if (!open[b]) continue;
            if (hs->skip[b] || swe[b] >= target[b]) {
                open[b] = false;
                // passes the block ran: queued ahead at the next step
                g->spec[b] = std::max(1, (hs->done[b] + g->spp[b] - 1) / g->spp[b]);
            } else {
                ahead[b] = enq[b] + 1;
            }
        }
    }
    if (!have) {
        const int rc = read_back();   // no block ran: the norms of dE' for the stats
        if (rc) return rc;
    }
    for (int q = 0; q < 3; q++) {
        const int b = c.ndim == 3 ? 0 : (q == 2 ? 1 : 0);
        if (hs->done[b] == 0) res[q] = (const T *)rhs[q];
        else res[q] = delta ? (const T *)g->S[q] : (const T *)g->X[hs->last[b]][q];
    }
    if (st) {
        for (int b = 0; b < 2; b++) {
            st->sweeps[b] = hs->done[b];
            st->resid[b] = hs->resid[b];
            st->rhs[b] = hs->rhsn[b];
            st->nonconverged[b] = active[b] && hs->done[b] > 0 && !hs->conv[b] ? 1 : 0;
        }
    }
    return MX_OK;
}

// Run the sweeps of one solve: x = sum_{j<count} A^j b per block (Alg 1).
// rhs: the right-hand side (dE' or Ebar).  Writes the per-block result
// pointers into res[3].  When E_fuse is set (fixed count), E += result is
// fused into a block's final pass and e_done[block] is set.  A tolerance
// solve (tolmode) is solve_tol's.
//
// The blocks of a 2D grid are independent: the row-streaming kernel runs the
// passes of each block on its own (groups {TE}, {TM}); the LDS-tile kernel
// and 3D run all blocks together (one group).  A group's count of sweeps is
// cut into the fewest passes of at most spp sweeps, of nearly equal depth
// (deeper ones last: the final pass also reads and writes E, so its sweeps
// are the cheapest).
// The front of a step when it runs fused with the first sweep pass
template <typename T>
struct FusedFront {
    FrontArgs<T> a;
    const T *Bin[3];
};

template <typename T>
int run_sweeps(mx_grid *g, void *const rhs[3], const int *target_in, bool tolmode, void *E_fuse[3],
               bool e_done[2], const T **res, mx_step_stats *st, const FusedFront<T> *ff = nullptr)
{
    e_done[0] = e_done[1] = false;
    if (tolmode) return solve_tol<T>(g, rhs, target_in, res, st);
    const mx_config &c = g->cfg;
    const Coef<T> &k = coef<T>(g);
    const int nblk = c.ndim == 3 ? 1 : 2;
    const bool cheb = c.solver == MX_SOLVER_CHEBYSHEV;
    const int form = cheb ? FM_CHEB : FM_STD;
    const bool split = c.ndim == 2 && g->variant == 3;
    int target[2] = {0, 0}, done[2] = {0, 0}, cur[2] = {-1, -1};
    bool fused[2] = {false, false};
    bool active_cfg[2];
    for (int b = 0; b < 2; b++) {
        active_cfg[b] = b < nblk && (c.ndim == 3 || (c.blocks & (1 << b)));
        target[b] = active_cfg[b] ? target_in[b] : 0;
    }
    if (cheb && (int)g->cheb[0][0].size() < std::max(target[0], target[1]))
        fill_cheb(&c, std::max(target[0], target[1]), g->cheb);
    const int groups[2] = {split ? 1 : 3, split ? 2 : 0};
    for (int gi = 0; gi < 2; gi++) {
        const int gmask = groups[gi];
        if (!gmask) continue;
        for (;;) {
            int act = 0, rem = 1 << 30;
            for (int b = 0; b < nblk; b++)
                if ((gmask & (1 << b)) && active_cfg[b] && done[b] < target[b]) {
                    act |= 1 << b;
                    rem = std::min(rem, target[b] - done[b]);
                }
            if (!act) break;
            const int spp = (act & 1) ? g->spp[0] : g->spp[1];
            const int kk = rem / ((rem + spp - 1) / spp);
            const bool first = (act & 1) ? done[0] == 0 : done[1] == 0;
            // E += x fused into this pass when every active block of the group ends here
            bool fin = E_fuse != nullptr;
            for (int b = 0; b < nblk; b++) {
                if (!(gmask & (1 << b)) || !active_cfg[b]) continue;
                if (!(act & (1 << b)) || done[b] + kk != target[b]) fin = false;
            }
            int flags = first ? SW_FIRST : 0;
            flags |= fin ? SW_LAST : SW_STORE;
            const int cb = (act & 1) ? cur[0] : cur[1];
            const int ob = cb == 0 ? 1 : 0;
            SweepArgs<T> a = pass_args<T>(g, rhs, cb, ob, first, cheb, E_fuse);
            if (cheb)
                for (int b = 0; b < 2; b++) pass_cheb<T>(g, b, done[b], kk, a);
            int nwg = 0;
            hipError_t e;
            if (ff && first) {
                // the front and this pass in one (the caller checked that the
                // pass is the first of both blocks and not the last)
                ProfScope ps(g, MX_PROF_FRONT_SWEEP, (double)g->ncell * sizeof(T) * (g->has_j ? 18 : 15));
                e = launch_front_sweep2d<T>(k, c.filter_passes, kk, ff->a, ff->Bin, a, g->stream, &nwg);
            } else {
                const int ncomp = c.ndim == 3 ? 3 : ((act & 1) ? 2 : 0) + ((act & 2) ? 1 : 0);
                ProfScope ps(g, fin ? MX_PROF_SWEEP_LAST : MX_PROF_SWEEP,
                             (double)g->ncell * sizeof(T) * pass_arrays(cheb, false, first, fin) * ncomp);
                if (c.ndim == 2 && g->variant == 1) e = launch_sweep2d<T>(k, act, kk, false, flags, a, g->stream, &nwg);
                else if (c.ndim == 2) e = launch_stream2d<T>(k, act, kk, form, flags, a, g->stream, &nwg, 0);
                else e = launch_sweep3d<T>(k, kk, form, flags, a, g->stream, &nwg);
            }
            if (e != hipSuccess) return fail(MX_EDEVICE, "sweep launch: %s", hipGetErrorString(e));
            for (int b = 0; b < nblk; b++)
                if (act & (1 << b)) { done[b] += kk; cur[b] = ob; fused[b] = fin; }
        }
    }
    for (int b = 0; b < 2; b++) e_done[b] = fused[b];
    for (int q = 0; q < 3; q++) {
        const int b = c.ndim == 3 ? 0 : (q == 2 ? 1 : 0);
        res[q] = done[b] == 0 ? (const T *)rhs[q] : (const T *)g->X[cur[b]][q];
    }
    if (st) {
        for (int b = 0; b < 2; b++) {
            st->sweeps[b] = done[b];
            st->resid[b] = 0.0;
            st->rhs[b] = 0.0;
            st->nonconverged[b] = 0;
        }
    }
    return MX_OK;
}

// The single-launch solve applies to 2D tolerance solves (Alg 1) on the
// LDS-tile kernel (grids too small for row streams) whose tiles fit the
// co-resident workgroups of one cooperative launch.
template <typename T>
bool small_ok(const mx_grid *g)
{
    const mx_config &c = g->cfg;
    if (c.ndim != 2 || !(c.tol > 0.0) || g->variant != 1 || c.solver != MX_SOLVER_ALG1 || c.lumped) return false;
    if (c.filter_passes > 4 || g->spp[0] < 1 || g->spp[0] > 8 || c.sweeps < 1 || !g->small_bar) return false;
    int ntx = 0, nty = 0;
    small_tiles<T>((int)c.n[0], (int)c.n[1], &ntx, &nty);
    return (long long)ntx * nty <= small_capacity<T>(c.form == MX_FORM_DELTA, c.blocks) && (long long)ntx * nty <= max_wg(&c);
}

template <typename T>
int small_steps(mx_grid *g, int nsteps, const double *env, mx_step_stats *stats)
{
    const mx_config &c = g->cfg;
    const bool delta = c.form == MX_FORM_DELTA;
    SmallArgs<T> a{};
    a.c = coef<T>(g);
    for (int q = 0; q < 3; q++) {
        a.E[q] = (T *)g->E[q];
        a.B[0][q] = (T *)(g->bloc[q] ? g->Bws[q] : g->B[q]);
        a.B[1][q] = (T *)(g->bloc[q] ? g->B[q] : g->Bws[q]);
        a.J0[q] = g->has_j ? (const T *)g->J0[q] : nullptr;
        a.dEp[q] = (T *)g->dEp[q];
        a.X[0][q] = (T *)g->X[0][q];
        a.X[1][q] = (T *)g->X[1][q];
        a.S[q] = (T *)g->S[q];
    }
    a.partial = g->partial;
    a.bar = g->small_bar;
    a.err = (int *)(g->small_bar + 3);
    a.stat = g->small_stat;
    a.env_src = (const T *)g->small_env;
    a.tol = c.tol;
    a.blocks = c.blocks;
    a.spp = g->spp[0];
    a.mmax = c.sweeps;
    a.filter_passes = g->has_j ? c.filter_passes : 0;
    small_tiles<T>((int)c.n[0], (int)c.n[1], &a.ntx, &a.nty);
    // host staging: the pinned buffer of mx_init grids, else the grid's own
    SmallStat *hs = g->hred ? (SmallStat *)g->hred : g->hstat;
    T *he = g->hred ? (T *)((char *)g->hred + SMALL_MAX_STEPS * sizeof(SmallStat)) : (T *)g->henv;
    static const unsigned zero[4] = {0, 0, 0, 0};
    for (int s0 = 0; s0 < nsteps; s0 += SMALL_MAX_STEPS) {
        const int n = std::min(SMALL_MAX_STEPS, nsteps - s0);
        for (int i = 0; i < n; i++) he[i] = (T)((env ? env[s0 + i] : 0.0) * c.four_pi * c.dt);
        HIPCHK(hipMemcpyAsync(g->small_env, he, n * sizeof(T), hipMemcpyHostToDevice, g->stream));
        HIPCHK(hipMemcpyAsync(g->small_bar, zero, 4 * sizeof(unsigned), hipMemcpyHostToDevice, g->stream));
        a.nsteps = n;
        {
            ProfScope ps(g, MX_PROF_SWEEP, 0.0);
            HIPCHK(launch_small<T>(a, delta, g->stream));
        }
        HIPCHK(hipMemcpyAsync(hs, g->small_stat, n * sizeof(SmallStat), hipMemcpyDeviceToHost, g->stream));
        unsigned flag[4];
        HIPCHK(hipMemcpyAsync(flag, g->small_bar, 4 * sizeof(unsigned), hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
        if (flag[3]) return fail(MX_EDEVICE, "single-launch tolerance solve: grid barrier timed out");
        for (int i = 0; i < n; i++) {
            if (hs[i].nonfinite & 1)
                return fail(MX_ENONFINITE, "step %lld: norm of dE' is not finite", (long long)(g->step + i));
            if (hs[i].nonfinite & 2)
                return fail(MX_ENONFINITE, "step %lld: a residual norm is not finite", (long long)(g->step + i));
            if (stats) {
                mx_step_stats &st = stats[s0 + i];
                for (int b = 0; b < 2; b++) {
                    st.sweeps[b] = hs[i].done[b];
                    st.resid[b] = hs[i].resid[b];
                    st.rhs[b] = hs[i].rhsn[b];
                    st.nonconverged[b] = (c.blocks & (1 << b)) && hs[i].done[b] > 0 && !hs[i].conv[b] ? 1 : 0;
                }
            }
        }
        // B of the active blocks moved to the other buffer after an odd count
        if (n & 1)
            for (int q = 0; q < 3; q++) {
                const bool act = q == 2 ? (c.blocks & 1) : (c.blocks & 2);
                if (!act) continue;
                std::swap(a.B[0][q], a.B[1][q]);
                g->bloc[q] ^= 1;
            }
        g->step += n;
    }
    return MX_OK;
}

template <typename T>
int step_impl(mx_grid *g, int nsteps, const double *env, const int *replay, mx_step_stats *stats)
{
    const mx_config &c = g->cfg;
    const Coef<T> &k = coef<T>(g);
    const int nblk = c.ndim == 3 ? 1 : 2;
    const bool tolmode = c.tol > 0.0 && replay == nullptr;
    if (tolmode && nsteps > 0 && small_ok<T>(g)) {
        const int rc = small_steps<T>(g, nsteps, env, stats);
        if (rc) return rc;
        nsteps = 0;   // done; the hand-back below returns B to the caller's buffers
    }
    for (int s = 0; s < nsteps; s++) {
        const double e = env ? env[s] : 0.0;
        const T env_src = (T)(e * c.four_pi * c.dt);
        int nwg = 0;
        int target[2];
        for (int b = 0; b < 2; b++) {
            target[b] = replay ? replay[2 * s + b] : c.sweeps;
            if (!replay && c.lumped) target[b] = 0;
            if (target[b] < 0) return fail(MX_EINVAL, "negative replayed sweep count at step %d", s);
        }
        // the front runs fused with the first sweep pass when both blocks
        // take the same count of Alg 1 sweeps in more than one pass and that
        // first pass's depth has a fused kernel
        FusedFront<T> ff{};
        bool fuse = false;
        if (c.ndim == 2 && g->variant == 4 && !tolmode && c.solver == MX_SOLVER_ALG1 && !c.lumped &&
            c.blocks == MX_ALL && target[0] == target[1] && target[0] > g->spp[0]) {
            const int m = target[0], kk = m / ((m + g->spp[0] - 1) / g->spp[0]);
            fuse = front_sweep2d_ok(c.dtype == MX_F64, kk, g->has_j ? c.filter_passes : 0);
        }
        if (c.ndim == 2) {
            const T *Bin[3];
            T *Bout[3];
            for (int q = 0; q < 3; q++) {
                Bin[q] = (const T *)(g->bloc[q] ? g->Bws[q] : g->B[q]);
                Bout[q] = (T *)(g->bloc[q] ? g->B[q] : g->Bws[q]);
            }
            FrontArgs<T> a{};
            for (int q = 0; q < 3; q++) {
                a.E[q] = (const T *)g->E[q];
                a.B[q] = Bout[q];
                a.J0[q] = g->has_j ? (const T *)g->J0[q] : nullptr;
                a.dEp[q] = (T *)g->dEp[q];
            }
            a.env_src = env_src;
            a.partial = tolmode ? g->partial : nullptr;
            if (fuse) {
                ff.a = a;
                for (int q = 0; q < 3; q++) ff.Bin[q] = Bin[q];
            }
            const double fb = (double)g->ncell * sizeof(T) *
                              (((c.blocks & 1) ? (g->has_j ? 8 : 6) : 0) + ((c.blocks & 2) ? (g->has_j ? 7 : 6) : 0));
            hipError_t er = hipSuccess;
            if (!fuse) {
                ProfScope ps(g, MX_PROF_FRONT, fb);
                er = launch_front_stream2d<T>(k, c.blocks, c.filter_passes, a, Bin, g->stream, &nwg);
            }
            if (er != hipSuccess) return fail(MX_EDEVICE, "front launch: %s", hipGetErrorString(er));
            // B components of active blocks now live in the other buffer
            if (c.blocks & 1) g->bloc[2] ^= 1;
            if (c.blocks & 2) { g->bloc[0] ^= 1; g->bloc[1] ^= 1; }
        } else if (c.filter_passes <= front3d_max_passes()) {
            // one pass: Faraday into the other B buffer, filter, dE'
            const T *Bin[3];
            FrontArgs<T> a{};
            for (int q = 0; q < 3; q++) {
                Bin[q] = (const T *)(g->bloc[q] ? g->Bws[q] : g->B[q]);
                a.B[q] = (T *)(g->bloc[q] ? g->B[q] : g->Bws[q]);
                a.E[q] = (const T *)g->E[q];
                a.J0[q] = g->has_j ? (const T *)g->J0[q] : nullptr;
                a.dEp[q] = (T *)g->dEp[q];
            }
            a.env_src = env_src;
            a.partial = tolmode ? g->partial : nullptr;
            hipError_t er;
            {
                ProfScope ps(g, MX_PROF_FRONT, (double)g->ncell * sizeof(T) * (g->has_j ? 15 : 12));
                er = launch_front3d<T>(k, c.filter_passes, a, Bin, g->stream, &nwg);
            }
            if (er != hipSuccess) return fail(MX_EDEVICE, "front launch: %s", hipGetErrorString(er));
            for (int q = 0; q < 3; q++) g->bloc[q] ^= 1;
        } else {
            hipError_t er;
            {
                ProfScope ps(g, MX_PROF_FRONT, (double)g->ncell * sizeof(T) * 9);
                er = launch_faraday3d<T>(k, (const T *const *)g->E, (T *const *)g->B, g->stream);
            }
            if (er != hipSuccess) return fail(MX_EDEVICE, "faraday launch: %s", hipGetErrorString(er));
            const T *const *jf = nullptr;
            if (g->has_j) {
                jf = (const T *const *)g->J0;
                if (c.filter_passes > 0) {
                    ProfScope ps(g, MX_PROF_FRONT, (double)g->ncell * sizeof(T) * 6 * 3 * c.filter_passes);
                    er = launch_filter3d<T>(k, c.filter_passes, (const T *const *)g->J0, (T *const *)g->Jf,
                                            (T *const *)g->Jt, g->stream);
                    if (er != hipSuccess) return fail(MX_EDEVICE, "filter launch: %s", hipGetErrorString(er));
                    jf = (const T *const *)g->Jf;
                }
            }
            {
                ProfScope ps(g, MX_PROF_FRONT, (double)g->ncell * sizeof(T) * (jf ? 9 : 6));
                er = launch_rhs3d<T>(k, (const T *const *)g->B, jf, env_src, (T *const *)g->dEp,
                                     tolmode ? g->partial : nullptr, g->stream, &nwg);
            }
            if (er != hipSuccess) return fail(MX_EDEVICE, "rhs launch: %s", hipGetErrorString(er));
        }
        if (tolmode) {
            // ||dE'|| per block starts the device-side state of the solve
            ProfScope ps(g, MX_PROF_OTHER, 0.0);
            HIPCHK(launch_reduce2(g->partial, nwg, g->red, g->stream));
            HIPCHK(launch_tol_init(g->tol, g->red, nblk, g->stream));
        }
        const T *res[3];
        bool e_done[2] = {false, false};
        mx_step_stats st{};
        int rc = run_sweeps<T>(g, g->dEp, target, tolmode, g->E, e_done, res, stats ? &st : nullptr,
                               fuse ? &ff : nullptr);
        if (rc) return rc;
        {
            // E += dE per block not fused into its last pass (the components
            // of inactive 2D blocks are left alone)
            for (int b = 0; b < nblk; b++) {
                if (c.ndim == 2 && !(c.blocks & (1 << b))) continue;
                if (e_done[b]) continue;
                const int mask = block_mask_comps(c.ndim, b);
                hipError_t er;
                {
                    ProfScope ps(g, MX_PROF_OTHER, (double)g->ncell * sizeof(T) * 3 * (mask == 7 ? 3 : mask == 3 ? 2 : 1));
                    er = launch_update<T>(g->ncell, mask, (T *const *)g->E, res, g->stream);
                }
                if (er != hipSuccess) return fail(MX_EDEVICE, "update launch: %s", hipGetErrorString(er));
            }
        }
        if (stats) stats[s] = st;
        g->step++;
    }
    // hand the state back in the caller's B buffers
    for (int q = 0; q < 3; q++)
        if (g->bloc[q]) {
            ProfScope ps(g, MX_PROF_OTHER, 2.0 * g->ncell * sizeof(T));
            HIPCHK(hipMemcpyAsync(g->B[q], g->Bws[q], (size_t)g->ncell * sizeof(T), hipMemcpyDeviceToDevice,
                                  g->stream));
            g->bloc[q] = 0;
        }
    return MX_OK;
}

template <typename T>
int adjoint_impl(mx_grid *g, int nsteps, const double *env, const int *sweeps, void *const Ebar[3],
                 void *const Bbar[3], void *const dJ0[3])
{
    const mx_config &c = g->cfg;
    const Coef<T> &k = coef<T>(g);
    const double arr = (double)g->ncell * sizeof(T);
    // The current gradient sum_n env_n (-4 pi dt) F v_n is F applied once to
    // sum_n env_n (-4 pi dt) v_n (F is linear): the steps accumulate the
    // unfiltered sum in a buffer the adjoint does not otherwise use (the B
    // workspace in 2D, the filtered-current buffer in 3D), filtered at the end
    T *const *acc = (T *const *)(c.ndim == 2 ? g->Bws : g->Jf);
    const int cmask = c.ndim == 3 ? 7 : ((c.blocks & 1) ? 3 : 0) | ((c.blocks & 2) ? 4 : 0);
    bool any_src = false;
    if (dJ0) {
        // all three components start at zero: a block the grid does not step
        // keeps a zero current gradient
        ProfScope ps(g, MX_PROF_ADJOINT, arr * 3);
        HIPCHK(launch_axpy3<T>(g->ncell, 7, true, T(0), acc, acc, g->stream));
    }
    for (int s = nsteps - 1; s >= 0; s--) {
        int target[2] = {sweeps[2 * s], sweeps[2 * s + 1]};
        const T *v[3];
        bool e_done[2] = {false, false};
        // v = P Ebar
        int rc = run_sweeps<T>(g, Ebar, target, false, nullptr, e_done, v, nullptr);
        if (rc) return rc;
        // Bbar += dt Lambda K v, with the current gradient's accumulator
        // acc += env (-4 pi dt) v in the same pass over v
        const double sc = -(env ? env[s] : 0.0) * c.four_pi * c.dt;
        const bool add = dJ0 && sc != 0.0;
        {
            const int ncomp = __builtin_popcount(cmask);
            ProfScope ps(g, MX_PROF_ADJOINT, arr * (9 + (add ? 2 * ncomp : 0)));
            HIPCHK(launch_adj_curlB<T>(k, c.ndim, c.blocks, v, (T *const *)Bbar, (T)sc, add ? acc : nullptr,
                                       g->stream));
        }
        any_src = any_src || add;
        {
            ProfScope ps(g, MX_PROF_ADJOINT, arr * 9);
            HIPCHK(launch_adj_curlE<T>(k, c.ndim, c.blocks, (const T *const *)Bbar, (T *const *)Ebar, g->stream));
        }
    }
    if (any_src) {
        // dJ0 += F acc; filter temporaries: dE' and the running-sum buffers
        ProfScope ps(g, MX_PROF_ADJOINT, arr * 3 * (2 * c.ndim * c.filter_passes + 3));
        HIPCHK(launch_adj_source<T>(k, c.ndim, c.filter_passes, (const T *const *)acc, (T *const *)g->dEp,
                                    (T *const *)g->S, T(1), (T *const *)dJ0, g->stream));
    }
    return MX_OK;
}

}  // namespace

extern "C" {

int mx_step(mx_grid *g, int nsteps, const double *env, const int *replay, mx_step_stats *stats)
{
    if (!g) return fail(MX_EINVAL, "grid is NULL");
    if (!g->bound) return fail(MX_ESTATE, "mx_step before mx_bind_fields");
    if (nsteps < 0) return fail(MX_EINVAL, "nsteps must be >= 0");
    HIPCHK(hipSetDevice(g->device));
    auto run = [&](mx_step_stats *st) {
        return g->cfg.dtype == MX_F64 ? step_impl<double>(g, nsteps, env, replay, st)
                                      : step_impl<float>(g, nsteps, env, replay, st);
    };
    const char *dump = std::getenv("MX_STATS");
    if (!dump || !*dump || std::strcmp(dump, "0") == 0) return run(stats);
    // per-step records as JSON lines: MX_STATS=1 writes them to stderr, any
    // other value names a file they are appended to
    std::vector<mx_step_stats> rec((size_t)nsteps);
    const int64_t s0 = g->step;
    const int rc = run(rec.data());
    const int done = (int)std::min<int64_t>(nsteps, g->step - s0);
    if (stats) std::copy(rec.begin(), rec.begin() + done, stats);
    FILE *f = std::strcmp(dump, "1") == 0 ? stderr : std::fopen(dump, "a");
    if (f) {
        const mx_config &c = g->cfg;
        for (int s = 0; s < done; s++) {
            const mx_step_stats &r = rec[s];
            std::fprintf(f,
                         "{\"grid\": \"%p\", \"step\": %lld, \"ndim\": %d, \"n\": [%lld, %lld, %lld], "
                         "\"tol\": %.6g, \"sweeps\": [%d, %d], \"resid\": [%.17g, %.17g], \"rhs\": [%.17g, %.17g], "
                         "\"nonconverged\": [%d, %d]}\n",
                         (void *)g, (long long)(s0 + s), c.ndim, (long long)c.n[0], (long long)c.n[1],
                         (long long)(c.ndim == 3 ? c.n[2] : 1), c.tol, r.sweeps[0], r.sweeps[1], r.resid[0],
                         r.resid[1], r.rhs[0], r.rhs[1], r.nonconverged[0], r.nonconverged[1]);
        }
        if (f != stderr) std::fclose(f);
    }
    return rc;
}

}  // extern "C"

namespace mx {
// nsteps steps of a grid laid out on the scratch `ws` (ws_bytes) of the
// current device, fields and current bound for this call only; allocates
// nothing: the grid descriptor lives on the stack, the tolerance read-back
// goes to pageable host memory, no timing events.  Alg 1 only (the
// Chebyshev factors are kept in host vectors).
int step_on_scratch(const mx_config *cfg, void *stream, int device, void *ws, size_t ws_bytes, void *const E[3],
                    void *const B[3], void *const J0[3], int nsteps, const double *env, const int *replay,
                    mx_step_stats *stats)
{
    int rc = mx_validate(cfg, nullptr);
    if (rc) return rc;
    if (cfg->solver != MX_SOLVER_ALG1)
        return fail(MX_EINVAL, "the static-scratch step runs Alg 1 only (the Chebyshev factors need host memory)");
    if (!E || !B) return fail(MX_EINVAL, "NULL argument");
    for (int q = 0; q < 3; q++) {
        if (!E[q] || !B[q]) return fail(MX_EINVAL, "field component %d is NULL", q);
        if (J0 && !J0[q]) return fail(MX_EINVAL, "J0 component %d is NULL", q);
    }
    if (nsteps < 0) return fail(MX_EINVAL, "nsteps must be >= 0");
    size_t need = 0;
    mx_workspace_size(cfg, &need);
    if (need > ws_bytes)
        return fail(MX_EWORKSPACE, "this grid needs %zu bytes of scratch; the static scratch holds %zu", need,
                    ws_bytes);
    mx_grid g;
    grid_setup(&g, cfg, (hipStream_t)stream, device, (char *)ws, ws_bytes);
    for (int q = 0; q < 3; q++) {
        g.E[q] = E[q];
        g.B[q] = B[q];
        g.J0[q] = J0 ? J0[q] : nullptr;
    }
    g.bound = true;
    g.has_j = J0 != nullptr;
    return cfg->dtype == MX_F64 ? step_impl<double>(&g, nsteps, env, replay, stats)
                                : step_impl<float>(&g, nsteps, env, replay, stats);
}
}  // namespace mx

extern "C" {

int mx_adjoint(mx_grid *g, int nsteps, const double *env, const int *sweeps, void *const Ebar[3],
               void *const Bbar[3], void *const dJ0[3])
{
    if (!g || !sweeps || !Ebar || !Bbar) return fail(MX_EINVAL, "NULL argument");
    if (nsteps < 0) return fail(MX_EINVAL, "nsteps must be >= 0");
    for (int q = 0; q < 3; q++)
        if (!Ebar[q] || !Bbar[q] || (dJ0 && !dJ0[q])) return fail(MX_EINVAL, "NULL component");
    for (int s = 0; s < 2 * nsteps; s++)
        if (sweeps[s] < 0) return fail(MX_EINVAL, "negative sweep count");
    HIPCHK(hipSetDevice(g->device));
    return g->cfg.dtype == MX_F64 ? adjoint_impl<double>(g, nsteps, env, sweeps, Ebar, Bbar, dJ0)
                                  : adjoint_impl<float>(g, nsteps, env, sweeps, Ebar, Bbar, dJ0);
}

}  // extern "C"

namespace {

template <typename T>
int pic_push_impl(mx_grid *g, int64_t np, double q, double m, double w, void *const pos[2], void *const u[3],
                  void *const J[3], bool zero_j)
{
    const mx_config &c = g->cfg;
    PicArgs<T> a{};
    for (int q3 = 0; q3 < 3; q3++) {
        a.E[q3] = (const T *)g->E[q3];
        a.B[q3] = (const T *)g->B[q3];
        a.J[q3] = (T *)J[q3];
    }
    a.x = (T *)(np ? pos[0] : nullptr);
    a.y = (T *)(np ? pos[1] : nullptr);
    a.ux = (T *)(np ? u[0] : nullptr);
    a.uy = (T *)(np ? u[1] : nullptr);
    a.uz = (T *)(np ? u[2] : nullptr);
    a.np = np;
    a.nx = (int)c.n[0];
    a.ny = (int)c.n[1];
    a.dx = (T)c.d[0];
    a.dy = (T)c.d[1];
    a.dt = (T)c.dt;
    a.th = (T)(0.5 * c.dt);
    a.h = (T)(q * c.dt / (2.0 * m));
    a.cx = (T)(-q * w / (c.d[1] * c.dt));
    a.cy = (T)(-q * w / (c.d[0] * c.dt));
    a.cz = (T)(q * w / (c.d[0] * c.d[1]));
    a.Lx = (T)(c.n[0] * c.d[0]);
    a.Ly = (T)(c.n[1] * c.d[1]);
    ProfScope ps(g, MX_PROF_PARTICLES, (double)np * sizeof(T) * 10);
    HIPCHK(launch_pic_push<T>(a, zero_j, g->stream));
    return MX_OK;
}

int pic_check(mx_grid *g, int64_t np)
{
    if (!g) return fail(MX_EINVAL, "grid is NULL");
    if (g->cfg.ndim != 2) return fail(MX_EINVAL, "the particle coupling is 2D");
    if (np < 0 || np > (int64_t)0x7fffffff * 256) return fail(MX_EINVAL, "np out of range");
    return MX_OK;
}

}  // namespace

extern "C" {

int mx_pic_push(mx_grid *g, int64_t np, double q, double m, double w, void *const pos[2], void *const u[3],
                void *const J[3], int accumulate)
{
    int rc = pic_check(g, np);
    if (rc) return rc;
    if (!g->bound) return fail(MX_ESTATE, "mx_pic_push before mx_bind_fields");
    if (g->cfg.blocks != MX_ALL) return fail(MX_EINVAL, "the particle push needs both 2D blocks (MX_ALL)");
    if (!(m > 0.0) || !std::isfinite(m) || !std::isfinite(q) || !std::isfinite(w))
        return fail(MX_EINVAL, "q, w must be finite and m positive");
    if (!J || !J[0] || !J[1] || !J[2]) return fail(MX_EINVAL, "J is NULL");
    if (np > 0) {
        if (!pos || !pos[0] || !pos[1] || !u || !u[0] || !u[1] || !u[2])
            return fail(MX_EINVAL, "particle arrays are NULL");
    }
    HIPCHK(hipSetDevice(g->device));
    return g->cfg.dtype == MX_F64 ? pic_push_impl<double>(g, np, q, m, w, pos, u, J, accumulate == 0)
                                  : pic_push_impl<float>(g, np, q, m, w, pos, u, J, accumulate == 0);
}

int mx_pic_charge(mx_grid *g, int64_t np, double q, double w, void *const pos[2], void *rho, int accumulate)
{
    int rc = pic_check(g, np);
    if (rc) return rc;
    if (!std::isfinite(q) || !std::isfinite(w)) return fail(MX_EINVAL, "q, w must be finite");
    if (!rho) return fail(MX_EINVAL, "rho is NULL");
    if (np > 0 && (!pos || !pos[0] || !pos[1])) return fail(MX_EINVAL, "positions are NULL");
    HIPCHK(hipSetDevice(g->device));
    const mx_config &c = g->cfg;
    const double cq = q * w / (c.d[0] * c.d[1]);
    const int nx = (int)c.n[0], ny = (int)c.n[1];
    if (c.dtype == MX_F64)
        HIPCHK(launch_pic_charge<double>(np, nx, ny, c.d[0], c.d[1], cq, np ? (const double *)pos[0] : nullptr,
                                         np ? (const double *)pos[1] : nullptr, (double *)rho, accumulate == 0,
                                         g->stream));
    else
        HIPCHK(launch_pic_charge<float>(np, nx, ny, (float)c.d[0], (float)c.d[1], (float)cq,
                                        np ? (const float *)pos[0] : nullptr, np ? (const float *)pos[1] : nullptr,
                                        (float *)rho, accumulate == 0, g->stream));
    return MX_OK;
}

int mx_sources_assemble(mx_grid *g, int nsrc, int W, const int64_t *origins, const void *shapes,
                        const void *amps, void *const J0[3])
{
    if (!g || !origins || !shapes || !amps || !J0) return fail(MX_EINVAL, "NULL argument");
    if (g->cfg.ndim != 2) return fail(MX_EINVAL, "source windows are 2D");
    if (nsrc < 0 || W < 1 || W > g->cfg.n[0] || W > g->cfg.n[1]) return fail(MX_EINVAL, "bad nsrc or W");
    HIPCHK(hipSetDevice(g->device));
    const int nx = (int)g->cfg.n[0], ny = (int)g->cfg.n[1];
    if (g->cfg.dtype == MX_F64)
        HIPCHK(launch_sources<double>(nx, ny, nsrc, W, origins, (const double *)shapes, (const double *)amps,
                                      (double *const *)J0, nullptr, nullptr, false, g->stream));
    else
        HIPCHK(launch_sources<float>(nx, ny, nsrc, W, origins, (const float *)shapes, (const float *)amps,
                                     (float *const *)J0, nullptr, nullptr, false, g->stream));
    return MX_OK;
}

int mx_sources_project(mx_grid *g, int nsrc, int W, const int64_t *origins, const void *shapes,
                       void *const G[3], void *grad)
{
    if (!g || !origins || !shapes || !G || !grad) return fail(MX_EINVAL, "NULL argument");
    if (g->cfg.ndim != 2) return fail(MX_EINVAL, "source windows are 2D");
    if (nsrc < 0 || W < 1 || W > g->cfg.n[0] || W > g->cfg.n[1]) return fail(MX_EINVAL, "bad nsrc or W");
    if (nsrc == 0) return MX_OK;
    HIPCHK(hipSetDevice(g->device));
    const int nx = (int)g->cfg.n[0], ny = (int)g->cfg.n[1];
    if (g->cfg.dtype == MX_F64)
        HIPCHK(launch_sources<double>(nx, ny, nsrc, W, origins, (const double *)shapes, nullptr, nullptr,
                                      (double *const *)G, (double *)grad, true, g->stream));
    else
        HIPCHK(launch_sources<float>(nx, ny, nsrc, W, origins, (const float *)shapes, nullptr, nullptr,
                                     (float *const *)G, (float *)grad, true, g->stream));
    return MX_OK;
}

}  // extern "C"
