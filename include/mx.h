/*
 * mx.h - C ABI of the MI355X field-step library for the unlumped
 * finite-element Maxwell solver of Lu et al., "An O(N) Maxwell solver with
 * improved numerical dispersion properties" (arXiv 1907.13088).
 *
 * One time step (Sec. 2.2.1, the update procedure after the A-matrix
 * equations) maps the state (E^n, B^{n-1/2}) to (E^{n+1}, B^{n+1/2}):
 *   1. B^{n+1/2} = B^{n-1/2} - c dt curl E^n          (eqs faraday_x..z)
 *   2. Jf = F^p (env_n J0), p binomial (1,2,1)/4 passes per axis; the
 *      paper filters the current (Sec. 4.2, Sec. 5) without naming a stencil
 *   3. dE' = c dt curl(Lambda B^{n+1/2}) - 4 pi dt Jf  (eqs ampere_aux_x..z)
 *   4. (1 - A) dE = dE' by the fixed-point sweeps of Alg 1,
 *      A from eqs matrixA_1st..matrixA_last (2D: matrixA_*_2d); in 2D
 *      optionally by the Chebyshev semi-iteration (MX_SOLVER_CHEBYSHEV)
 *   5. E^{n+1} = E^n + dE
 * with c = 1, periodic boundaries in every axis.
 *
 * Memory model.  The caller owns the device memory of every grid: field
 * buffers are borrowed device pointers and the library's scratch lives in a
 * caller-provided workspace of mx_workspace_size() bytes.  The library never
 * allocates device memory at run time (mx_init takes 80 bytes of pinned host
 * memory, to read the tolerance solve's state back); its one static device
 * array, the scratch of mx_step_static (MX_STATIC_SCRATCH_BYTES per GPU),
 * comes with the loaded code.  All kernels run on the HIP stream given to
 * mx_init (NULL = the default stream).
 *
 * Layout.  Each field component is one dense array in the grid dtype
 * (float or double), x fastest: index (k*ny + j)*nx + i, nz = 1 in 2D.
 * Components sit at the paper's staggered positions (variable list, Sec. 2):
 *   Ex (i+1/2, j, k)  Ey (i, j+1/2, k)  Ez (i, j, k+1/2)
 *   Bx (i, j+1/2, k+1/2)  By (i+1/2, j, k+1/2)  Bz (i+1/2, j+1/2, k)
 *   J like E.  E is at time level n, B at n - 1/2 (B first, then E).
 *
 * Errors.  Every call returns MX_OK (0) or a negative code; the message of
 * the calling thread's last failure is given by mx_last_error().  Argument
 * errors are detected on the host before any device work.  Non-convergence
 * of a tolerance solve is not an error: it is flagged in mx_step_stats.
 */
#ifndef MX_H
#define MX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MX_OK            0
#define MX_EINVAL       -1   /* bad argument: NULL, size, enum, layout */
#define MX_ECFL         -2   /* dt above the stability limit (Sec. 2.1) */
#define MX_EWORKSPACE   -3   /* workspace missing or smaller than required */
#define MX_EDEVICE      -4   /* HIP runtime error */
#define MX_ENONFINITE   -5   /* a residual norm became NaN or Inf */
#define MX_ESTATE       -6   /* call out of order (e.g. step before bind) */

#define MX_F32 0
#define MX_F64 1

/* decoupled blocks: in 2D TE = (Ex, Ey, Bz) and TM = (Ez, Bx, By) evolve
   independently (Sec. 2.2.2); 3D always uses MX_ALL */
#define MX_TE  1
#define MX_TM  2
#define MX_ALL 3

/* iterate form of the tolerance solve (a reading, not in the paper):
   STANDARD keeps x_(j+1) = dE' + A x_(j) (Alg 1); DELTA keeps
   d_(j+1) = A d_(j) and s_(j+1) = s_(j) + d_(j+1), identical in exact
   arithmetic, whose step norm |d| has no FP32 rounding floor */
#define MX_FORM_STANDARD 0
#define MX_FORM_DELTA    1

/* solve of the mass-matrix system (1 - A) dE = dE' (eq transform-e-e_aux):
   ALG1 is the paper's fixed-point iteration (Alg 1, Sec. 2.2.1); CHEBYSHEV
   is the Chebyshev semi-iteration on each 2D block's spectral interval of
   1 - A, [1 - rho, 1] with rho = 2/3 (TE) and the largest corner value of
   the TM symbol, an accelerated solve the paper names as future work
   (Sec. 2.2.1).  It counts sweeps like Alg 1 (one application of A each)
   and its tolerance test uses the same residual ||dE' + A x - x||_2, but
   its iterates differ: it reaches a given residual in far fewer sweeps.
   2D row streaming (variants 0, 2, 3) or 3D with cubic cells (where 1 - A
   spans [1/9, 1]); standard form, not lumped; not in a batch.  Its result
   after m sweeps is a polynomial in A applied to dE', so mx_adjoint
   transposes it with the same kernels. */
#define MX_SOLVER_ALG1      0
#define MX_SOLVER_CHEBYSHEV 1

/* init-time warnings (bit flags) */
#define MX_WARN_NOCONV_GUARANTEE 1  /* 3D, dt > min(d)/sqrt(2): the infinity-norm
                                       convergence bound of Appendix C does not hold */

typedef struct mx_config {
    int ndim;             /* 2 or 3 */
    int64_t n[3];         /* cells per axis; n[2] ignored (1) in 2D */
    double d[3];          /* cell sizes dx, dy, dz (> 0) */
    double dt;            /* time step, c = 1; must satisfy the CFL bound */
    int dtype;            /* MX_F32 or MX_F64 */
    int blocks;           /* 2D: MX_TE, MX_TM or MX_ALL; 3D: MX_ALL */
    int sweeps;           /* m when tol == 0; m_max when tol > 0 (>= 0) */
    double tol;           /* 0: fixed m (the paper's choice, Sec. 2.2.1);
                             > 0: stop when ||dE_(j+1) - dE_(j)||_2 <= tol ||dE'||_2
                             per block, tested after every pass of sweeps */
    int filter_passes;    /* p >= 0 */
    int lumped;           /* 1: averaging operators lumped, the Yee scheme (Sec. 2) */
    double four_pi;       /* source constant, 4 pi in Gaussian units */
    int form;             /* MX_FORM_STANDARD or MX_FORM_DELTA */
    int sweeps_per_pass;  /* sweeps fused per pass over HBM, in [0, 16]; 0 = library
                             choice.  Row streaming (2D) caps it at the deepest
                             kernel built: both blocks together 9 (FP32), 4 (FP64),
                             delta form 8, 3; per block TE 14 (FP32), 7 (FP64),
                             delta 12, 6; TM 16 (FP32), 12 (FP64), delta 16, 10.
                             LDS tile: <= 8.
                             3D: up to 3 in FP32, 2 in FP64 (library choice: the
                             most allowed). */
    int variant;          /* 2D sweep kernel: 0 library choice (FP32: 4, FP64 and
                             the Chebyshev solve: 3; Alg 1 on a grid whose
                             streaming pass would have fewer workgroups than
                             half the CUs: 1),
                             1 LDS tile (both blocks per pass; by default 5
                             sweeps deep in FP32, 4 in FP64, 8 under a
                             tolerance), 2 row streaming
                             (both blocks per pass), 3 row streaming (each block
                             on its own), 4 as 2 with the front (Faraday,
                             filter, dE') run in the same pass as the first
                             sweeps (FP32, fixed m of Alg 1 in more than one
                             pass, m / ceil(m / spp) in 3..6, p <= 4; other
                             steps run as in 2) */
    int solver;           /* MX_SOLVER_ALG1 (default) or MX_SOLVER_CHEBYSHEV (2D,
                             and 3D with cubic cells); the
                             2D Chebyshev passes fuse at most: both blocks 6
                             (FP32), 2 (FP64); TE 10, 4; TM 16, 8 */
} mx_config;

typedef struct mx_step_stats {
    int sweeps[2];        /* sweeps taken per block (2D: TE, TM; 3D: [0]) */
    double resid[2];      /* last step norm ||dE_(j+1) - dE_(j)||_2 (tol mode;
                             the Chebyshev solve: the residual ||dE' + A x - x||_2
                             of its last sweep's input, the same quantity) */
    double rhs[2];        /* ||dE'||_2 (tol mode) */
    int nonconverged[2];  /* tol mode: m_max reached above tolerance */
} mx_step_stats;

typedef struct mx_grid mx_grid;

/* Thread-local message of the last failed call ("" if none). */
const char *mx_last_error(void);

/* Fill *cfg with defaults: 2D, unit cells, FP32, MX_ALL, m = 20, tol = 0,
   no filter, 4 pi, standard form, Alg 1.  n and dt must still be set. */
int mx_config_default(mx_config *cfg);

/* Host-only validation (no device call): ranges, enums and the CFL bound
   dt <= (sum_i 1/d_i^2)^(-1/2) (Sec. 2.1).  *warn receives MX_WARN_* bits
   (may be NULL). */
int mx_validate(const mx_config *cfg, int *warn);

/* Bytes of device workspace mx_init needs for cfg (host-only). */
int mx_workspace_size(const mx_config *cfg, size_t *bytes);

/* Create a grid.  `stream` is a hipStream_t (NULL = default stream);
   `workspace` a device buffer of at least mx_workspace_size() bytes, owned
   by the caller and kept alive until mx_destroy.  Validates like
   mx_validate.  Sets the current device to the one `workspace` is on. */
int mx_init(const mx_config *cfg, void *stream, void *workspace, size_t workspace_bytes,
            mx_grid **out);

/* Bind the state: E[3] at level n and B[3] at level n - 1/2, borrowed
   device pointers in the grid dtype and layout (updated in place). */
int mx_bind_fields(mx_grid *g, void *const E[3], void *const B[3]);

/* Bind the prescribed current shape J0[3] (device pointers, layout of E,
   borrowed, read only); J0 == NULL removes the source. */
int mx_set_current(mx_grid *g, void *const J0[3]);

/* Advance nsteps steps.  env (host, nsteps doubles, may be NULL = 0)
   scales J0 at step s, i.e. at t = (n + s + 1/2) dt.  replay (host,
   2*nsteps ints, may be NULL) forces the per-block sweep counts of each
   step instead of the configured rule.  stats (host, nsteps entries, may
   be NULL) receives per-step counts and norms.  Asynchronous on the stream
   unless tol > 0: then the stop test runs on the device after every pass,
   passes are queued ahead of it (as many per block as the previous step
   needed; those after convergence do nothing) and the call waits about
   once per step to read the outcome; a non-finite norm is reported at
   that read. */
int mx_step(mx_grid *g, int nsteps, const double *env, const int *replay, mx_step_stats *stats);
/* (With the environment variable MX_STATS set, mx_step also writes each
   step's record as one JSON line: MX_STATS=1 to stderr, any other value
   names a file the lines are appended to; "0" or empty: off.) */

/* Step counter n of the bound state. */
int mx_get_step(mx_grid *g, int64_t *n);
int mx_set_step(mx_grid *g, int64_t n);

/* Sweeps fused per HBM pass in use (the library's or the configured choice):
   that of the TE block when it is active, else that of TM.  With a fixed m
   a block's m sweeps run in the fewest passes of at most this depth, of
   nearly equal depth, the deeper ones last; under a tolerance the stop
   test follows every pass, and both 2D blocks then use one depth unless
   sweeps_per_pass is capped. */
int mx_get_sweeps_per_pass(mx_grid *g, int *k);

/* Sweeps per pass of each 2D block: k[0] TE, k[1] TM (3D: k[0]). */
int mx_get_block_sweeps_per_pass(mx_grid *g, int k[2]);

int mx_destroy(mx_grid *g);

/* ------------------------------------------------------------------------
 * Allocation-free stepping, for callers that cannot allocate memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  mx_step_static runs nsteps steps like mx_init + mx_bind_fields
 * + mx_set_current + mx_step, with the same arguments and results, but its
 * scratch (the workspace of mx_workspace_size) is a device array of
 * MX_STATIC_SCRATCH_BYTES inside this library, one per GPU, held until the
 * process ends: the call allocates no device or host memory and keeps no
 * state between calls.  It runs on the current device, whose copy of the
 * array it looks up on its first call there.
 *   cfg      as for mx_init; Alg 1 only (MX_SOLVER_ALG1)
 *   stream   hipStream_t (NULL = default stream)
 *   E, B     the state (device pointers, grid layout), updated in place
 *   J0       the current shape (device pointers) or NULL
 *   nsteps, env, replay, stats   as for mx_step
 * A config whose mx_workspace_size exceeds MX_STATIC_SCRATCH_BYTES is
 * rejected with MX_EWORKSPACE before any device work (64 MiB hold, e.g., a
 * 1024^2 FP32 or a 512 x 1024 FP64 2D grid).  Every call on one GPU uses the
 * same array: calls that overlap on one GPU (other host threads, other
 * streams) race and give wrong results; serialise them.  The array keeps
 * the last call's contents; every value a step reads from it is written
 * earlier in the same step, so nothing needs clearing between calls.
 * ------------------------------------------------------------------------ */
#define MX_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int mx_step_static(const mx_config *cfg, void *stream, void *const E[3], void *const B[3], void *const J0[3],
                   int nsteps, const double *env, const int *replay, mx_step_stats *stats);

/* ------------------------------------------------------------------------
 * Per-kernel timing.  While enabled, every launch of mx_step / mx_adjoint is
 * bracketed by HIP events recorded on the grid's stream, and its algorithmic
 * HBM traffic (each array a kernel must read or write, counted once per
 * touched cell) is added to its category.  mx_profile_enable(g, 1) resets
 * the counters and starts recording, (g, 0) pauses (the counters are kept),
 * (g, 2) resumes without a reset, so that a caller can sample some steps of
 * a longer run; mx_profile_read waits for the stream and sums the event
 * times recorded since the last reset.
 * ------------------------------------------------------------------------ */
#define MX_PROF_FRONT      0  /* filter + Faraday + auxiliary increment */
#define MX_PROF_SWEEP      1  /* mass-matrix sweep passes that store the iterate */
#define MX_PROF_OTHER      2  /* separate E increments, FP64 reductions, copies */
#define MX_PROF_ADJOINT    3  /* transposed curls and the filter of the adjoint */
#define MX_PROF_SWEEP_LAST 4  /* final sweep passes with E += result fused */
#define MX_PROF_PARTICLES  5  /* particle push and deposition (bytes: the phase space read and written) */
#define MX_PROF_FRONT_SWEEP 6 /* the front fused with the first sweep pass (2D variant 4) */
#define MX_PROF_NCAT       7
typedef struct mx_profile {
    int64_t launches[MX_PROF_NCAT];
    double ms[MX_PROF_NCAT];     /* summed kernel time per category */
    double bytes[MX_PROF_NCAT];  /* summed algorithmic bytes per category */
} mx_profile;

int mx_profile_enable(mx_grid *g, int on);
int mx_profile_read(mx_grid *g, mx_profile *out);

/* ------------------------------------------------------------------------
 * Transposed (adjoint) step.  The step is linear in (E, B, J0):
 *   B+ = B - dt K E,   E+ = E + P (dt K^T Lambda B+ - 4 pi dt env F J0),
 * K the E->B curl of eqs faraday_*, K^T the B->E curl of eqs ampere_aux_*,
 * Lambda = diag(alpha_x, alpha_y, alpha_z), P = sum_{j<=m} A^j (Alg 1; the
 * Chebyshev solve's P is its polynomial in A after m sweeps) and F the filter.  A is symmetric (Appendix C), as are Lambda and F, so the
 * transposed step is
 *   v = P Ebar;  Bbar += dt Lambda K v;  Ebar -= dt K^T Bbar;
 *   dJ0 += env (-4 pi dt) F v.
 * mx_adjoint runs nsteps transposed steps in reverse order for forward steps
 * n0 .. n0+nsteps-1: env[s] and sweeps[2s], sweeps[2s+1] are those of
 * forward step n0+s.  Ebar, Bbar (device, grid layout, in: gradient with
 * respect to the state after the steps, out: before) are updated in place;
 * dJ0 (device, may be NULL) accumulates the gradient with respect to J0.
 * Uses the grid's workspace; the bound fields are not touched.
 * ------------------------------------------------------------------------ */
int mx_adjoint(mx_grid *g, int nsteps, const double *env, const int *sweeps,
               void *const Ebar[3], void *const Bbar[3], void *const dJ0[3]);

/* ------------------------------------------------------------------------
 * Particle coupling (2D grids, three velocity components).  The paper runs
 * the field solver inside a particle-in-cell code and keeps that code's
 * force interpolation, current deposition and particle push (Sec. 2); with
 * a charge-conserving deposition Gauss's law for E is kept (Sec. 2,
 * Appendix A).  A coupled step is: mx_pic_push for every species (J^{n+1/2}
 * from the moves), then mx_step(g, 1, env = {1.0}, ...) with J0 bound to J
 * (mx_set_current), which filters it and advances the fields.
 *
 * mx_pic_push: one push of np particles of charge q, mass m (> 0) and
 * weight w (macro-particle: charge q w) in the bound E^n and
 * B^n = B^{n-1/2} - (dt/2) curl E^n, by the relativistic Boris scheme
 * (Boris 1970; c = 1), fields interpolated with first-order B-spline shapes
 * at each component's staggered position (the lowest order of Table 1);
 * then the move and Esirkepov's charge-conserving deposition (Esirkepov
 * 2001) of J^{n+1/2}, so that rho^{n+1} - rho^n + dt D.J^{n+1/2} = 0 at the
 * nodes.  pos[2] = x, y (device, np values in the grid dtype; physical
 * coordinates, node (i, j) at (i dx, j dy), in [0, L); in: n, out: n + 1,
 * wrapped), u[3] = gamma v (in: n - 1/2, out: n + 1/2).  J[3] (device,
 * placed like E) is overwritten (accumulate = 0) or added to (1, further
 * species).  J is a current density per cell area.  A particle moves less
 * than a cell per step: |v| < 1 and dt obeys the CFL bound.  The
 * deposition adds with floating-point atomics: J is reproducible up to the
 * order of those additions (rounding).  Needs blocks = MX_ALL; the bound
 * fields are read, not changed.
 *
 * mx_pic_charge: rho at the nodes (i, j) (device, grid dtype) of the same
 * particles, the density whose change the deposition's current carries;
 * overwritten (accumulate = 0) or added to.
 * ------------------------------------------------------------------------ */
int mx_pic_push(mx_grid *g, int64_t np, double q, double m, double w, void *const pos[2], void *const u[3],
                void *const J[3], int accumulate);
int mx_pic_charge(mx_grid *g, int64_t np, double q, double w, void *const pos[2], void *rho, int accumulate);

/* ------------------------------------------------------------------------
 * Localised 2D source shapes.  Source s has three W x W windows
 * shapes[((s*3 + c)*W + a)*W + b] (device, grid dtype) whose cell (a, b)
 * lands on grid cell ((x0_s + b) mod nx, (y0_s + a) mod ny), with
 * origins[2s] = x0_s, origins[2s+1] = y0_s (device int64).
 *   mx_sources_assemble:  J0 = sum_s amps[s] shape_s   (J0 overwritten)
 *   mx_sources_project:   grad[s] = <shape_s, G>        (the transpose)
 * amps and grad are device arrays of nsrc values in the grid dtype.
 * ------------------------------------------------------------------------ */
int mx_sources_assemble(mx_grid *g, int nsrc, int W, const int64_t *origins, const void *shapes,
                        const void *amps, void *const J0[3]);
int mx_sources_project(mx_grid *g, int nsrc, int W, const int64_t *origins, const void *shapes,
                       void *const G[3], void *grad);

/* ------------------------------------------------------------------------
 * Batched stepping of independent 2D periodic grids (each its own size,
 * dt and coefficients; TE+TM; no current; one fixed m >= 1 for all grids;
 * one dtype).  Every phase of a step of all grids is one launch over the
 * concatenated work items of the batch; with persistent = 1 all nsteps
 * steps of all grids run inside a single cooperative launch, in which
 * workgroups claim the work items of all steps and phases in order from an
 * atomic counter and an item waits only until the previous phase of its own
 * grid has completed (per-grid counters; no grid-wide barrier, so the items
 * of other grids fill the tail of a phase); the wait is bounded (a
 * time-out returns MX_EDEVICE).  In FP32 the front and the first sweep
 * pass of a step run as one phase when that pass is 3..6 sweeps deep and
 * not the last (both schedules).  Passes are at most sweeps_per_pass of the
 * first config deep (capped at 7); mx_batch_init with sweeps_per_pass = 0
 * times candidate pass depths and chunk lengths on workspace scratch
 * fields (the bound state is never touched), separately for the grouped
 * and the persistent schedule, and keeps the fastest of each.  The chosen
 * plans are kept in a text file and reused by a later init of the same
 * grid configs on the same device and library build: $MX_TUNE_CACHE (a
 * path; "0" or empty turns the cache off), else
 * $XDG_CACHE_HOME/mx/batch_plans.txt or $HOME/.cache/mx/batch_plans.txt.
 * The workspace holds 15 arrays per grid.
 * ------------------------------------------------------------------------ */
typedef struct mx_batch mx_batch;

int mx_batch_workspace_size(const mx_config *cfgs, int ngrids, size_t *bytes);
int mx_batch_init(const mx_config *cfgs, int ngrids, void *stream, void *workspace,
                  size_t workspace_bytes, mx_batch **out);
int mx_batch_bind(mx_batch *b, int grid, void *const E[3], void *const B[3]);
int mx_batch_step(mx_batch *b, int nsteps, int persistent);
/* The schedules in use: sweeps per pass of the grouped schedule (tuned at
   init when the configs ask for sweeps_per_pass = 0), its total work items
   of one step, and the workgroups of the persistent launch. */
int mx_batch_get_plan(mx_batch *b, int *sweeps_per_pass, int *tiles_total, int *persistent_blocks);
/* One schedule's tuned shape (persistent = 0 grouped, 1 persistent): the
   deepest pass (sweeps), the rows of a sweep work item's chunk and of a
   front work item's, and the work items of one step (front plus sweep
   passes; in FP32 the front and the first pass run as one phase on the
   front's items when that pass is 3..6 sweeps deep and not the last).  Any output pointer may be NULL.  Host only; MX_EINVAL for a
   NULL batch. */
int mx_batch_get_schedule(mx_batch *b, int persistent, int *sweeps_per_pass, int *chunk_rows, int *front_rows,
                          int *items_per_step);
int mx_batch_destroy(mx_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* MX_H */
