// Host side of the batched 2D stepping entry points (mx_batch_* in mx.h):
// validation, workspace carving, device descriptors, the grouped and the
// persistent schedules, and the autotuner for sweeps per pass and chunk
// length.
#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <queue>
#include <string>
#include <vector>

#include "mx_internal.h"

using namespace mx;

namespace mx {
int api_fail(int code, const char *msg);   // mx_api.cpp
}

namespace {

constexpr size_t ALIGN = 256;
size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

int bfail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return api_fail(code, buf);
}

#define BCHK(expr)                                                                              \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return bfail(MX_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// full-grid arrays per grid: dE' (3), two iterates (6), second B (3), scratch
// fields the autotuner times on (3)
constexpr int ARRAYS = 15;

int64_t cells(const mx_config &c) { return c.n[0] * c.n[1]; }

template <typename T>
void fill_coef2(const mx_config &c, Coef<T> &k)
{
    const double dt = c.dt, dx = c.d[0], dy = c.d[1];
    const double rx = dt * dt / (dx * dx), ry = dt * dt / (dy * dy), rxy = dt * dt / (dx * dy);
    std::memset(&k, 0, sizeof(k));
    k.nx = (int)c.n[0];
    k.ny = (int)c.n[1];
    k.nz = 1;
    k.tdx = (T)(dt / dx);
    k.tdy = (T)(dt / dy);
    k.tdz = (T)dt;
    k.src = (T)(c.four_pi * dt);
    k.cxx = (T)((ry - 1.0) / 6.0);
    k.cyy = (T)((rx - 1.0) / 6.0);
    k.cxy = (T)(-rxy / 6.0);
    k.czx = (T)((rx - 1.0) / 6.0);
    k.czy = (T)((ry - 1.0) / 6.0);
    k.czz = (T)((rx + ry - 1.0) / 36.0);
    k.lumped = 0;
}

}  // namespace

struct mx_batch {
    int ng;
    int dtype;
    int m;
    hipStream_t stream;
    int device;
    std::vector<mx_config> cfg;
    std::vector<int64_t> ncell;
    std::vector<void *> E, B;          // 3 per grid (caller's)
    std::vector<void *> ws;            // ARRAYS per grid
    std::vector<int> bound;
    void *desc;                        // device GridDesc<T>[ng]
    int *items_f, *items_s;            // device prefix sums (ng + 1)
    unsigned *cnt;                     // device: claim counter, then per-grid phase counters
    int ncnt;                          // per-grid phase counters available (ng * (m + 1))
    int *err;                          // device error flag
    int spp, Lf, Ls;                   // grouped schedule: pass depth cap, chunk rows
    int pk, pLf, pLs;                  // persistent schedule: the same
    int nf, ns;                        // items per phase (of the last upload)
    bool tuned;
};

namespace {

// pass sizes of one step: the fewest passes of at most k sweeps, sizes as
// equal as possible, the deeper ones last (as the single-grid schedule)
void pass_sizes(int m, int k, std::vector<int> &sz)
{
    sz.clear();
    const int np = (m + k - 1) / k;
    const int q = m / np, r = m % np;
    for (int p = 0; p < np; p++) sz.push_back(p >= np - r ? q + 1 : q);
}

// column width the sweep work items are cut with: the narrowest strip of
// any pass depth the schedule runs (a strip of a wider pass then covers its
// columns with room to spare; a narrower one would leave columns out)
int cut_width(int m, int k)
{
    std::vector<int> sz;
    pass_sizes(m, k, sz);
    int w = 1 << 30;
    for (int s : sz) w = std::min(w, batch2d::sweep_width(s));
    return w;
}

// persistent passes: npass passes, the first nlow of q - 1 sweeps, the rest q
void persistent_shape(int m, int k, int *q, int *npass, int *nlow)
{
    std::vector<int> sz;
    pass_sizes(m, k, sz);
    *npass = (int)sz.size();
    *q = sz.back();
    *nlow = 0;
    for (int v : sz) *nlow += v < *q ? 1 : 0;
}

template <typename T>
int upload(mx_batch *b, bool scratch_fields, int k, int Lf, int Ls)
{
    // Descriptors and item tables for a schedule of passes at most k deep
    // and chunks of Lf (front) and Ls (sweeps) rows.  With scratch_fields
    // the E and B of every grid point at workspace arrays (the autotuner's
    // trial steps never touch the caller's state).
    std::vector<GridDesc<T>> d(b->ng);
    std::vector<int> itf(b->ng + 1, 0), its(b->ng + 1, 0);
    const int wf = batch2d::front_width(), wsw = cut_width(b->m, k);
    for (int g = 0; g < b->ng; g++) {
        const mx_config &c = b->cfg[g];
        GridDesc<T> &gd = d[g];
        std::memset(&gd, 0, sizeof(gd));
        fill_coef2(c, gd.c);
        T **w = (T **)&b->ws[(size_t)g * ARRAYS];
        for (int q = 0; q < 3; q++) {
            gd.dEp[q] = w[q];
            gd.X[0][q] = w[3 + q];
            gd.X[1][q] = w[6 + q];
            gd.B[1][q] = w[9 + q];
            if (scratch_fields) {
                gd.E[q] = w[12 + q];
                gd.B[0][q] = w[3 + q];   // the first iterate buffer doubles as old B
            } else {
                gd.E[q] = (T *)b->E[3 * g + q];
                gd.B[0][q] = (T *)b->B[3 * g + q];
            }
        }
        const int nx = (int)c.n[0], ny = (int)c.n[1];
        gd.nsx_f = (nx + wf - 1) / wf;
        gd.nsx_s = (nx + wsw - 1) / wsw;
        itf[g + 1] = itf[g] + gd.nsx_f * ((ny + Lf - 1) / Lf);
        its[g + 1] = its[g] + gd.nsx_s * ((ny + Ls - 1) / Ls);
    }
    b->nf = itf[b->ng];
    b->ns = its[b->ng];
    BCHK(hipMemcpyAsync(b->desc, d.data(), sizeof(GridDesc<T>) * b->ng, hipMemcpyHostToDevice, b->stream));
    BCHK(hipMemcpyAsync(b->items_f, itf.data(), sizeof(int) * (b->ng + 1), hipMemcpyHostToDevice, b->stream));
    BCHK(hipMemcpyAsync(b->items_s, its.data(), sizeof(int) * (b->ng + 1), hipMemcpyHostToDevice, b->stream));
    BCHK(hipStreamSynchronize(b->stream));   // the host vectors go out of scope
    return MX_OK;
}

// the front runs fused with the first pass (FP32, more than one pass, a
// first pass of 3..6 sweeps: the depths the fused kernel is built for)
template <typename T>
bool fuse_first(int first, int npass)
{
    return sizeof(T) == 4 && npass >= 2 && first >= batch2d::FUSE_KMIN && first <= batch2d::FUSE_KMAX;
}

template <typename T>
int grouped_steps(mx_batch *b, int nsteps, int bin0)
{
    const GridDesc<T> *d = (const GridDesc<T> *)b->desc;
    std::vector<int> sz;
    pass_sizes(b->m, b->spp, sz);
    const bool fuse = fuse_first<T>(sz[0], (int)sz.size());
    int bin = bin0;
    for (int s = 0; s < nsteps; s++) {
        if (fuse)
            BCHK(batch2d::launch_front_sweep<T>(d, b->ng, b->items_f, b->nf, b->Lf, sz[0], bin, b->stream));
        else
            BCHK(batch2d::launch_front<T>(d, b->ng, b->items_f, b->nf, b->Lf, bin, b->stream));
        bin ^= 1;
        for (size_t p = fuse ? 1 : 0; p < sz.size(); p++) {
            const bool first = p == 0, last = p + 1 == sz.size();
            BCHK(batch2d::launch_sweep<T>(d, b->ng, b->items_s, b->ns, b->Ls, sz[p], first, last,
                                          (int)((p + 1) & 1), (int)(p & 1), b->stream));
        }
    }
    return MX_OK;
}

template <typename T>
int persistent_steps(mx_batch *b, int nsteps, int bin0)
{
    int q, npass, nlow;
    persistent_shape(b->m, b->pk, &q, &npass, &nlow);
    const int fuse = fuse_first<T>(nlow > 0 ? q - 1 : q, npass) ? 1 : 0;
    const int nph = 1 + npass - fuse;   // phases per step
    // the claim counter runs over a whole launch: at most 2^31 - 1 items
    const long long per_step = (long long)b->nf + (long long)(npass - fuse) * b->ns;
    const int max_steps = (int)std::max(1LL, std::min<long long>(0x7fffffffLL, 0x7fffffffLL / per_step));
    // the error flag starts at zero (a copy: no memset node in a captured
    // stream); a time-out flagged in one launch makes the later ones leave
    // at their first wait
    static const int zero = 0;
    BCHK(hipMemcpyAsync(b->err, &zero, sizeof(int), hipMemcpyHostToDevice, b->stream));
    for (int s0 = 0; s0 < nsteps; s0 += max_steps) {
        const int n = std::min(max_steps, nsteps - s0);
        BCHK(batch2d::launch_persistent<T>((const GridDesc<T> *)b->desc, b->ng, b->items_f, b->items_s, b->pLf,
                                           b->pLs, n, q, npass, nlow, bin0 ^ (s0 & 1), b->cnt, b->ng * nph, b->err,
                                           fuse, b->stream));
    }
    int h = 0;
    BCHK(hipMemcpyAsync(&h, b->err, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    BCHK(hipStreamSynchronize(b->stream));
    if (h) return bfail(MX_EDEVICE, "persistent batch launch: a wait for the previous phase timed out");
    return MX_OK;
}

// Time four steps of each candidate plan (pass depth cap x chunk rows) on
// scratch fields, for the grouped and for the persistent schedule.
// Modelled length, in row steps, of one sweep pass of a batch whose work
// items are cut into chunks of L rows for passes at most k deep: each of
// `slots` resident workgroups claims the next item as it finishes (list
// scheduling in item order), and an item of r output rows takes r + 3k
// steps (its pipeline fills and drains k rows per level).  Long chunks pay
// the fill less often; the item count decides how evenly the last items
// spread over the workgroups.
double chunk_makespan(const mx_batch *b, int k, int L, int slots)
{
    const int w = cut_width(b->m, k);
    std::priority_queue<double, std::vector<double>, std::greater<double>> busy;
    for (int i = 0; i < slots; i++) busy.push(0.0);
    double end = 0.0;
    for (const mx_config &c : b->cfg) {
        const int nx = (int)c.n[0], ny = (int)c.n[1];
        const int nsx = (nx + w - 1) / w;
        for (int y0 = 0; y0 < ny; y0 += L)
            for (int sx = 0; sx < nsx; sx++) {
                const double t = busy.top() + std::min(L, ny - y0) + 3 * k;
                busy.pop();
                busy.push(t);
                end = std::max(end, t);
            }
    }
    return end;
}

// chunk lengths to time for passes at most k deep: a fixed set plus the
// three the model above ranks best (multiples of 8 from 32 to 512)
std::vector<int> chunk_candidates(const mx_batch *b, int k, int slots)
{
    std::vector<int> ls = {64, 128, 256};
    std::vector<std::pair<double, int>> ranked;
    for (int L = 32; L <= 512; L += 8) ranked.push_back({chunk_makespan(b, k, L, slots), L});
    std::sort(ranked.begin(), ranked.end());
    for (int i = 0, added = 0; i < (int)ranked.size() && added < 3; i++)
        if (std::find(ls.begin(), ls.end(), ranked[i].second) == ls.end()) {
            ls.push_back(ranked[i].second);
            added++;
        }
    return ls;
}

// two timing events, destroyed on every return path
struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~EventPair()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

template <typename T>
int autotune(mx_batch *b, bool grouped, bool persistent)
{
    EventPair ev;
    BCHK(hipEventCreate(&ev.e0));
    BCHK(hipEventCreate(&ev.e1));
    const hipEvent_t e0 = ev.e0, e1 = ev.e1;
    // FP32 passes fit two waves per SIMD up to 7 sweeps, FP64 up to 3
    const std::vector<int> ks = sizeof(T) == 4 ? std::vector<int>{4, 5, 6, 7} : std::vector<int>{2, 3, 4};
    for (int sched = 0; sched < 2; sched++) {
        if ((sched == 0 && !grouped) || (sched == 1 && !persistent)) continue;
        float best = 1e30f;
        int bk = 5, bl = 64;
        for (int k : ks) {
            int q, npass, nlow;
            persistent_shape(b->m, k, &q, &npass, &nlow);
            // resident workgroups: the persistent grid (the grouped
            // schedule's sweep kernels have the same occupancy)
            const int slots = batch2d::persistent_blocks<T>(q);
            for (int l : chunk_candidates(b, k, slots > 0 ? slots : 512)) {
                int rc = upload<T>(b, true, k, l, l);
                if (rc) return rc;
                const int keep[6] = {b->spp, b->Lf, b->Ls, b->pk, b->pLf, b->pLs};
                b->spp = b->pk = k;
                b->Lf = b->Ls = b->pLf = b->pLs = l;
                rc = sched == 0 ? grouped_steps<T>(b, 1, 0) : persistent_steps<T>(b, 1, 0);   // warm
                if (!rc) {
                    BCHK(hipEventRecord(e0, b->stream));
                    rc = sched == 0 ? grouped_steps<T>(b, 4, 0) : persistent_steps<T>(b, 4, 0);
                    BCHK(hipEventRecord(e1, b->stream));
                }
                b->spp = keep[0]; b->Lf = keep[1]; b->Ls = keep[2];
                b->pk = keep[3]; b->pLf = keep[4]; b->pLs = keep[5];
                if (rc) return rc;
                BCHK(hipEventSynchronize(e1));
                float ms = 0.f;
                BCHK(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) { best = ms; bk = k; bl = l; }
            }
        }
        // the front phase's chunk rows on their own, with the chosen sweeps
        int blf = bl;
        for (int lf : {64, 128, 256}) {
            if (lf == bl) continue;
            int rc = upload<T>(b, true, bk, lf, bl);
            if (rc) return rc;
            const int keep[6] = {b->spp, b->Lf, b->Ls, b->pk, b->pLf, b->pLs};
            b->spp = b->pk = bk;
            b->Lf = b->pLf = lf;
            b->Ls = b->pLs = bl;
            rc = sched == 0 ? grouped_steps<T>(b, 1, 0) : persistent_steps<T>(b, 1, 0);   // warm
            if (!rc) {
                BCHK(hipEventRecord(e0, b->stream));
                rc = sched == 0 ? grouped_steps<T>(b, 4, 0) : persistent_steps<T>(b, 4, 0);
                BCHK(hipEventRecord(e1, b->stream));
            }
            b->spp = keep[0]; b->Lf = keep[1]; b->Ls = keep[2];
            b->pk = keep[3]; b->pLf = keep[4]; b->pLs = keep[5];
            if (rc) return rc;
            BCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            BCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) { best = ms; blf = lf; }
        }
        if (sched == 0) { b->spp = bk; b->Lf = blf; b->Ls = bl; }
        else { b->pk = bk; b->pLf = blf; b->pLs = bl; }
    }
    return MX_OK;
}

// Tuned schedules are kept on disk, one line per batch shape:
//   <key> <spp> <Lf> <Ls> <pk> <pLf> <pLs>
// The key hashes the grid configs (sizes, cells, dt, dtype, m), the device
// (architecture name, compute units) and this library's build, so a plan
// is reused only where it was measured.  The file is $MX_TUNE_CACHE when
// set ("0" or empty: no cache), else $XDG_CACHE_HOME/mx/batch_plans.txt or
// $HOME/.cache/mx/batch_plans.txt.  A missing or unreadable file only
// means the autotuner runs.
std::string tune_cache_path()
{
    const char *e = std::getenv("MX_TUNE_CACHE");
    if (e) return (e[0] == '\0' || std::strcmp(e, "0") == 0) ? std::string() : std::string(e);
    std::string dir;
    if (const char *x = std::getenv("XDG_CACHE_HOME")) dir = x;
    else if (const char *h = std::getenv("HOME")) dir = std::string(h) + "/.cache";
    else return std::string();
    dir += "/mx";
    (void)mkdir(dir.c_str(), 0755);
    return dir + "/batch_plans.txt";
}

uint64_t tune_key(const mx_batch *b)
{
    uint64_t h = 1469598103934665603ULL;   // FNV-1a
    auto mix = [&](const void *p, size_t n) {
        for (size_t i = 0; i < n; i++) { h ^= ((const unsigned char *)p)[i]; h *= 1099511628211ULL; }
    };
    const char *build = __DATE__ " " __TIME__;
    mix(build, std::strlen(build));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) {
        mix(prop.gcnArchName, std::strlen(prop.gcnArchName));
        mix(&prop.multiProcessorCount, sizeof(prop.multiProcessorCount));
    }
    mix(&b->ng, sizeof(b->ng));
    mix(&b->dtype, sizeof(b->dtype));
    mix(&b->m, sizeof(b->m));
    for (const mx_config &c : b->cfg) {
        mix(c.n, sizeof(c.n));
        mix(c.d, sizeof(c.d));
        mix(&c.dt, sizeof(c.dt));
    }
    return h;
}

bool tune_cache_load(mx_batch *b, const std::string &path, uint64_t key)
{
    if (path.empty()) return false;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    char line[256];
    bool hit = false;
    while (std::fgets(line, sizeof(line), f)) {
        unsigned long long k = 0;
        int v[6];
        if (std::sscanf(line, "%llx %d %d %d %d %d %d", &k, &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) != 7) continue;
        if (k != key) continue;
        bool ok = v[0] >= 1 && v[0] <= batch2d::KMAX && v[3] >= 1 && v[3] <= batch2d::KMAX;
        for (int i : {1, 2, 4, 5}) ok = ok && v[i] >= 8 && v[i] <= 4096;
        if (!ok) continue;
        b->spp = v[0]; b->Lf = v[1]; b->Ls = v[2];
        b->pk = v[3]; b->pLf = v[4]; b->pLs = v[5];
        hit = true;   // the last matching line wins
    }
    std::fclose(f);
    return hit;
}

void tune_cache_store(const mx_batch *b, const std::string &path, uint64_t key)
{
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%016llx %d %d %d %d %d %d\n", (unsigned long long)key, b->spp, b->Lf, b->Ls, b->pk, b->pLf,
                 b->pLs);
    std::fclose(f);
}

}  // namespace

extern "C" {

int mx_batch_workspace_size(const mx_config *cfgs, int ngrids, size_t *bytes)
{
    if (!cfgs || !bytes || ngrids < 1) return bfail(MX_EINVAL, "bad batch arguments");
    size_t tot = 0;
    for (int g = 0; g < ngrids; g++) {
        const mx_config &c = cfgs[g];
        int rc = mx_validate(&c, nullptr);
        if (rc) return rc;
        if (c.ndim != 2 || c.blocks != MX_ALL || c.tol != 0.0 || c.lumped || c.sweeps < 1 || c.dtype != cfgs[0].dtype
            || c.sweeps != cfgs[0].sweeps || c.solver != MX_SOLVER_ALG1)
            return bfail(MX_EINVAL, "grid %d: a batch holds 2D TE+TM grids of one dtype, one fixed m >= 1, "
                                    "Alg 1, no lumping", g);
        tot += ARRAYS * up((size_t)cells(c) * (c.dtype == MX_F64 ? 8 : 4));
    }
    const size_t dsz = cfgs[0].dtype == MX_F64 ? sizeof(GridDesc<double>) : sizeof(GridDesc<float>);
    tot += up(dsz * ngrids) + 2 * up(sizeof(int) * (ngrids + 1)) + up(sizeof(int));
    tot += up(sizeof(unsigned) * (1 + (size_t)ngrids * (cfgs[0].sweeps + 1)));
    *bytes = tot;
    return MX_OK;
}

int mx_batch_init(const mx_config *cfgs, int ngrids, void *stream, void *workspace, size_t workspace_bytes,
                  mx_batch **out)
{
    if (!out) return bfail(MX_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    int rc = mx_batch_workspace_size(cfgs, ngrids, &need);
    if (rc) return rc;
    if (!workspace || workspace_bytes < need)
        return bfail(MX_EWORKSPACE, "batch workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, need);
    if (((uintptr_t)workspace) % ALIGN) return bfail(MX_EINVAL, "workspace must be %zu-byte aligned", ALIGN);
    hipPointerAttribute_t attr;
    BCHK(hipPointerGetAttributes(&attr, workspace));
    if (attr.type != hipMemoryTypeDevice) return bfail(MX_EINVAL, "workspace is not device memory");
    BCHK(hipSetDevice(attr.device));
    // owned here until the batch is complete: every early return frees it
    std::unique_ptr<mx_batch> hold(new mx_batch());
    mx_batch *b = hold.get();
    b->ng = ngrids;
    b->dtype = cfgs[0].dtype;
    b->m = cfgs[0].sweeps;
    b->stream = (hipStream_t)stream;
    b->device = attr.device;
    b->cfg.assign(cfgs, cfgs + ngrids);
    b->E.assign(3 * ngrids, nullptr);
    b->B.assign(3 * ngrids, nullptr);
    b->bound.assign(ngrids, 0);
    char *p = (char *)workspace;
    const size_t el = b->dtype == MX_F64 ? 8 : 4;
    for (int g = 0; g < ngrids; g++) {
        b->ncell.push_back(cells(cfgs[g]));
        const size_t arr = up((size_t)b->ncell[g] * el);
        for (int a = 0; a < ARRAYS; a++) { b->ws.push_back(p); p += arr; }
    }
    // zero the field arrays so trial steps never see stale bit patterns
    const size_t field_bytes = (size_t)(p - (char *)workspace);
    BCHK(hipMemsetAsync(workspace, 0, field_bytes, b->stream));
    const size_t dsz = b->dtype == MX_F64 ? sizeof(GridDesc<double>) : sizeof(GridDesc<float>);
    b->desc = p; p += up(dsz * ngrids);
    b->items_f = (int *)p; p += up(sizeof(int) * (ngrids + 1));
    b->items_s = (int *)p; p += up(sizeof(int) * (ngrids + 1));
    b->err = (int *)p; p += up(sizeof(int));
    b->cnt = (unsigned *)p;
    b->ncnt = ngrids * (b->m + 1);
    b->spp = b->pk = cfgs[0].sweeps_per_pass > 0 ? std::min(cfgs[0].sweeps_per_pass, batch2d::KMAX) : 5;
    b->Lf = b->Ls = b->pLf = b->pLs = 64;
    b->tuned = false;
    if (cfgs[0].sweeps_per_pass == 0) {
        const std::string path = tune_cache_path();
        const uint64_t key = tune_key(b);
        if (!tune_cache_load(b, path, key)) {
            rc = b->dtype == MX_F64 ? autotune<double>(b, true, true) : autotune<float>(b, true, true);
            if (rc) return rc;
            tune_cache_store(b, path, key);
        }
        b->tuned = true;
    }
    *out = hold.release();
    return MX_OK;
}

int mx_batch_bind(mx_batch *b, int grid, void *const E[3], void *const B[3])
{
    if (!b || !E || !B || grid < 0 || grid >= b->ng) return bfail(MX_EINVAL, "bad batch bind arguments");
    for (int q = 0; q < 3; q++) {
        if (!E[q] || !B[q]) return bfail(MX_EINVAL, "field component %d of grid %d is NULL", q, grid);
        b->E[3 * grid + q] = E[q];
        b->B[3 * grid + q] = B[q];
    }
    b->bound[grid] = 1;
    return MX_OK;
}

int mx_batch_step(mx_batch *b, int nsteps, int persistent)
{
    if (!b) return bfail(MX_EINVAL, "batch is NULL");
    if (nsteps < 0) return bfail(MX_EINVAL, "nsteps must be >= 0");
    for (int g = 0; g < b->ng; g++)
        if (!b->bound[g]) return bfail(MX_ESTATE, "grid %d of the batch is not bound", g);
    if (nsteps == 0) return MX_OK;
    BCHK(hipSetDevice(b->device));
    const bool f64 = b->dtype == MX_F64;
    int rc;
    if (persistent) {
        rc = f64 ? upload<double>(b, false, b->pk, b->pLf, b->pLs) : upload<float>(b, false, b->pk, b->pLf, b->pLs);
        if (!rc) rc = f64 ? persistent_steps<double>(b, nsteps, 0) : persistent_steps<float>(b, nsteps, 0);
    } else {
        rc = f64 ? upload<double>(b, false, b->spp, b->Lf, b->Ls) : upload<float>(b, false, b->spp, b->Lf, b->Ls);
        if (!rc) rc = f64 ? grouped_steps<double>(b, nsteps, 0) : grouped_steps<float>(b, nsteps, 0);
    }
    if (rc) return rc;
    // after an odd number of steps B lives in the workspace: hand it back
    if (nsteps % 2 == 1) {
        for (int g = 0; g < b->ng; g++)
            for (int q = 0; q < 3; q++)
                BCHK(hipMemcpyAsync(b->B[3 * g + q], b->ws[(size_t)g * ARRAYS + 9 + q], b->ncell[g] * (f64 ? 8 : 4),
                                    hipMemcpyDeviceToDevice, b->stream));
    }
    return MX_OK;
}

int mx_batch_get_plan(mx_batch *b, int *sweeps_per_pass, int *tiles_total, int *persistent_blocks)
{
    if (!b) return bfail(MX_EINVAL, "batch is NULL");
    if (sweeps_per_pass) *sweeps_per_pass = b->spp;
    if (tiles_total) {
        int rc = b->dtype == MX_F64 ? upload<double>(b, true, b->spp, b->Lf, b->Ls)
                                    : upload<float>(b, true, b->spp, b->Lf, b->Ls);
        if (rc) return rc;
        *tiles_total = b->nf + b->ns;
    }
    if (persistent_blocks) {
        int q, npass, nlow;
        persistent_shape(b->m, b->pk, &q, &npass, &nlow);
        *persistent_blocks = b->dtype == MX_F64 ? batch2d::persistent_blocks<double>(q)
                                                : batch2d::persistent_blocks<float>(q);
    }
    return MX_OK;
}

int mx_batch_get_schedule(mx_batch *b, int persistent, int *sweeps_per_pass, int *chunk_rows, int *front_rows,
                          int *items_per_step)
{
    if (!b) return bfail(MX_EINVAL, "batch is NULL");
    const int k = persistent ? b->pk : b->spp, Lf = persistent ? b->pLf : b->Lf, Ls = persistent ? b->pLs : b->Ls;
    if (sweeps_per_pass) *sweeps_per_pass = k;
    if (chunk_rows) *chunk_rows = Ls;
    if (front_rows) *front_rows = Lf;
    if (items_per_step) {
        // front items (with the first pass when it runs fused), then one
        // set of sweep items per other pass
        std::vector<int> sz;
        pass_sizes(b->m, k, sz);
        const bool f64 = b->dtype == MX_F64;
        const size_t nsep = sz.size() - ((f64 ? fuse_first<double>(sz[0], (int)sz.size())
                                              : fuse_first<float>(sz[0], (int)sz.size())) ? 1 : 0);
        const int wf = batch2d::front_width(), ws = cut_width(b->m, k);
        long long n = 0;
        for (const mx_config &c : b->cfg) {
            const long long nx = c.n[0], ny = c.n[1];
            n += ((nx + wf - 1) / wf) * ((ny + Lf - 1) / Lf);
            n += (long long)nsep * ((nx + ws - 1) / ws) * ((ny + Ls - 1) / Ls);
        }
        *items_per_step = (int)std::min<long long>(n, 0x7fffffff);
    }
    return MX_OK;
}

int mx_batch_destroy(mx_batch *b)
{
    delete b;
    return MX_OK;
}

}  // extern "C"
