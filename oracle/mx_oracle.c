/*
 * FP64 CPU oracle for one time step of the unlumped finite-element Maxwell
 * solver of Lu et al. (arXiv 1907.13088).  TEST INFRASTRUCTURE ONLY: it is
 * used by the tests, by the package smoke check and by the CPU baseline leg
 * of the benchmark, never by the product path.  It shares no code with the
 * HIP library.
 *
 * Plain scalar loops over periodic grids, written from the paper:
 *   Faraday update ........ eqs faraday_x..z (Sec. 2), 2D forms in Sec. 2.2.2
 *   auxiliary increment ... eqs ampere_aux_x..z (Sec. 2.2.1), 2D in Sec. 2.2.2
 *   mass-matrix system .... eq transform-e-e_aux with A from eqs
 *                           matrixA_1st..matrixA_last (3D) and
 *                           matrixA_1st_2d..matrixA_last_2d (2D)
 *   fixed-point solve ..... Alg 1 (Sec. 2.2.1)
 *   accelerated solve ..... optional Chebyshev semi-iteration on each 2D
 *                           block's spectral interval (the paper names faster
 *                           solves as future work; see ora_solve)
 *   E increment ........... E^{n+1} = E^n + dE (Sec. 2.2.1)
 *   low-pass filter ....... applied to the current (Sec. 4.2, Sec. 5); the
 *                           paper gives no stencil, the reading taken is p
 *                           passes of the binomial (1,2,1)/4 per axis.
 * Readings where the paper is silent: c = 1; the state is (E^n, B^{n-1/2});
 * j acts at n+1/2; a tolerance stop uses the relative L2 norm of successive
 * iterates per decoupled block, accumulated in FP64.
 *
 * Array layout: f[(k*ny + j)*nx + i], x fastest, periodic in every axis.
 * Component positions follow the paper's staggered variable list (Sec. 2):
 * Ex (i+1/2,j,k), Ey (i,j+1/2,k), Ez (i,j,k+1/2), Bx (i,j+1/2,k+1/2),
 * By (i+1/2,j,k+1/2), Bz (i+1/2,j+1/2,k); J like E.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int ndim;            /* 2 or 3 */
    long nx, ny, nz;     /* nz = 1 in 2D */
    double dx, dy, dz;
    double dt;           /* c = 1, so tau = c dt = dt */
    int blocks;          /* 2D: bit0 TE (Ex,Ey,Bz), bit1 TM (Ez,Bx,By); 3D: 3 */
    int sweeps;          /* m (tol == 0) or m_max (tol > 0) */
    double tol;          /* 0: fixed number of sweeps */
    int check_every;     /* a tolerance stop is tested after every g-th sweep */
    int filter_passes;   /* p */
    int lumped;          /* all averaging operators -> 1: the Yee scheme */
    double four_pi;      /* source constant */
    int solver;          /* 0: Alg 1; 1: Chebyshev semi-iteration (see ora_solve) */
} ora_cfg;

typedef struct {
    int sweeps[2];       /* per block (2D: TE, TM; 3D: [0]) */
    double resid[2];     /* last ||dE_(j+1) - dE_(j)||_2 per block */
    double rhs[2];       /* ||dE'||_2 per block */
    int nonconverged[2];
} ora_stats;

static inline long wrap(long i, long n)
{
    if (i >= 0 && i < n) return i;
    i %= n;
    return i < 0 ? i + n : i;
}

#define IDX(c, i, j, k) (((wrap((k), (c)->nz) * (c)->ny + wrap((j), (c)->ny)) * (c)->nx) + wrap((i), (c)->nx))

static long ncell(const ora_cfg *c) { return c->nx * c->ny * c->nz; }

/* averaging operator alpha along one axis (Sec. 2): (f- + 4 f + f+)/6 */
static inline double avg3(double fm, double f0, double fp, int lumped)
{
    return lumped ? f0 : (fm + 4.0 * f0 + fp) / 6.0;
}

/* ------------------------------------------------------------------------ */
/* Faraday: B^{n+1/2} = B^{n-1/2} - c dt curl E^n  (eqs faraday_x..z)       */
/* ------------------------------------------------------------------------ */
void ora_faraday(const ora_cfg *c, double *const E[3], double *B[3])
{
    const double t = c->dt;
    const int d3 = (c->ndim == 3);
    #pragma omp parallel for collapse(2)
    for (long k = 0; k < c->nz; k++)
        for (long j = 0; j < c->ny; j++)
            for (long i = 0; i < c->nx; i++) {
                long o = IDX(c, i, j, k);
                /* D_y Ez, D_z Ey at Bx (i, j+1/2, k+1/2) */
                double dyEz = (E[2][IDX(c, i, j + 1, k)] - E[2][o]) / c->dy;
                double dzEy = d3 ? (E[1][IDX(c, i, j, k + 1)] - E[1][o]) / c->dz : 0.0;
                /* D_z Ex, D_x Ez at By (i+1/2, j, k+1/2) */
                double dzEx = d3 ? (E[0][IDX(c, i, j, k + 1)] - E[0][o]) / c->dz : 0.0;
                double dxEz = (E[2][IDX(c, i + 1, j, k)] - E[2][o]) / c->dx;
                /* D_x Ey, D_y Ex at Bz (i+1/2, j+1/2, k) */
                double dxEy = (E[1][IDX(c, i + 1, j, k)] - E[1][o]) / c->dx;
                double dyEx = (E[0][IDX(c, i, j + 1, k)] - E[0][o]) / c->dy;
                if (c->ndim == 3 || (c->blocks & 2)) {
                    B[0][o] -= t * (dyEz - dzEy);
                    B[1][o] -= t * (dzEx - dxEz);
                }
                if (c->ndim == 3 || (c->blocks & 1))
                    B[2][o] -= t * (dxEy - dyEx);
            }
}

/* ------------------------------------------------------------------------ */
/* Low-pass filter on the current: p passes of (1,2,1)/4 along x, y (and z) */
/* ------------------------------------------------------------------------ */
void ora_filter(const ora_cfg *c, const double *src, double *dst)
{
    long n = ncell(c);
    double *tmp = (double *)malloc(sizeof(double) * n);
    memcpy(dst, src, sizeof(double) * n);
    for (int p = 0; p < c->filter_passes; p++) {
        for (int ax = 0; ax < c->ndim; ax++) {
            memcpy(tmp, dst, sizeof(double) * n);
            #pragma omp parallel for collapse(2)
            for (long k = 0; k < c->nz; k++)
                for (long j = 0; j < c->ny; j++)
                    for (long i = 0; i < c->nx; i++) {
                        long di = ax == 0, dj = ax == 1, dk = ax == 2;
                        dst[IDX(c, i, j, k)] = 0.25 * tmp[IDX(c, i - di, j - dj, k - dk)]
                                             + 0.5 * tmp[IDX(c, i, j, k)]
                                             + 0.25 * tmp[IDX(c, i + di, j + dj, k + dk)];
                    }
        }
    }
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Auxiliary increment (eqs ampere_aux_x..z):                               */
/*   dE' = c dt curl(Lambda B^{n+1/2}) - 4 pi dt Jf,                        */
/* Lambda = diag(alpha_x, alpha_y, alpha_z) acting on (Bx, By, Bz).         */
/* Jf may be NULL (no current).                                             */
/* ------------------------------------------------------------------------ */
void ora_rhs(const ora_cfg *c, double *const B[3], double *const Jf[3], double src_scale,
             double *dEp[3])
{
    const double t = c->dt;
    const int L = c->lumped;
    const int d3 = (c->ndim == 3);
    #pragma omp parallel for collapse(2)
    for (long k = 0; k < c->nz; k++)
        for (long j = 0; j < c->ny; j++)
            for (long i = 0; i < c->nx; i++) {
                long o = IDX(c, i, j, k);
                const double *Bx = B[0], *By = B[1], *Bz = B[2];
                /* alpha_z Bz at (i+1/2, j+1/2, k) and at j-1 / i-1 */
#define AZBZ(ii, jj) (d3 ? avg3(Bz[IDX(c, ii, jj, k - 1)], Bz[IDX(c, ii, jj, k)], Bz[IDX(c, ii, jj, k + 1)], L) : Bz[IDX(c, ii, jj, k)])
#define AYBY(ii, kk) avg3(By[IDX(c, ii, j - 1, kk)], By[IDX(c, ii, j, kk)], By[IDX(c, ii, j + 1, kk)], L)
#define AXBX(jj, kk) avg3(Bx[IDX(c, i - 1, jj, kk)], Bx[IDX(c, i, jj, kk)], Bx[IDX(c, i + 1, jj, kk)], L)
                /* x: D_y(alpha_z Bz) - D_z(alpha_y By) at Ex (i+1/2, j, k) */
                double cx = (AZBZ(i, j) - AZBZ(i, j - 1)) / c->dy;
                if (d3) cx -= (AYBY(i, k) - AYBY(i, k - 1)) / c->dz;
                /* y: D_z(alpha_x Bx) - D_x(alpha_z Bz) at Ey (i, j+1/2, k) */
                double cy = -(AZBZ(i, j) - AZBZ(i - 1, j)) / c->dx;
                if (d3) cy += (AXBX(j, k) - AXBX(j, k - 1)) / c->dz;
                /* z: D_x(alpha_y By) - D_y(alpha_x Bx) at Ez (i, j, k+1/2) */
                double cz = (AYBY(i, k) - AYBY(i - 1, k)) / c->dx
                          - (AXBX(j, k) - AXBX(j - 1, k)) / c->dy;
#undef AZBZ
#undef AYBY
#undef AXBX
                double s = c->four_pi * c->dt * src_scale;
                dEp[0][o] = t * cx - (Jf ? s * Jf[0][o] : 0.0);
                dEp[1][o] = t * cy - (Jf ? s * Jf[1][o] : 0.0);
                dEp[2][o] = t * cz - (Jf ? s * Jf[2][o] : 0.0);
            }
}

/* ------------------------------------------------------------------------ */
/* y = A x for the components in `mask` (bit q = component q), eqs          */
/* matrixA_*.  D-bar_i is the undivided difference f_{i+1/2} - f_{i-1/2};   */
/* D-bar_ii the second difference; (1 + D-bar_zz/6) is alpha_z.             */
/* ------------------------------------------------------------------------ */
void ora_apply_A(const ora_cfg *c, double *const x[3], double *y[3], int mask)
{
    const double t2 = c->dt * c->dt;
    const double rx = t2 / (c->dx * c->dx), ry = t2 / (c->dy * c->dy);
    const double rz = c->ndim == 3 ? t2 / (c->dz * c->dz) : 0.0;
    const double rxy = t2 / (c->dx * c->dy);
    const double ryz = c->ndim == 3 ? t2 / (c->dy * c->dz) : 0.0;
    const double rzx = c->ndim == 3 ? t2 / (c->dz * c->dx) : 0.0;
    const int d3 = (c->ndim == 3);
    #pragma omp parallel for collapse(2)
    for (long k = 0; k < c->nz; k++)
        for (long j = 0; j < c->ny; j++)
            for (long i = 0; i < c->nx; i++) {
                long o = IDX(c, i, j, k);
                const double *X = x[0], *Y = x[1], *Z = x[2];
#define F(a, ii, jj, kk) a[IDX(c, ii, jj, kk)]
                /* second differences of a component along one axis */
#define DXX(a, ii, jj, kk) (F(a, ii + 1, jj, kk) - 2.0 * F(a, ii, jj, kk) + F(a, ii - 1, jj, kk))
#define DYY(a, ii, jj, kk) (F(a, ii, jj + 1, kk) - 2.0 * F(a, ii, jj, kk) + F(a, ii, jj - 1, kk))
#define DZZ(a, ii, jj, kk) (F(a, ii, jj, kk + 1) - 2.0 * F(a, ii, jj, kk) + F(a, ii, jj, kk - 1))
                if (mask & 1) {
                    /* A_xx Ex: ((ry-1)/6) Dyy + ((rz-1)/6) Dzz + ((ry+rz-1)/36) Dyyzz */
                    double v = (ry - 1.0) / 6.0 * DYY(X, i, j, k);
                    if (d3) v += (rz - 1.0) / 6.0 * DZZ(X, i, j, k)
                               + (ry + rz - 1.0) / 36.0 * (DZZ(X, i, j + 1, k) - 2.0 * DZZ(X, i, j, k) + DZZ(X, i, j - 1, k));
                    /* A_xy Ey = -(t^2/(6 dx dy)) Dx Dy (1 + Dzz/6) Ey: Ey (i,j+1/2,k) -> Ex (i+1/2,j,k) */
                    double axy = 0.0;
                    for (int dk = -1; dk <= 1; dk++) {
                        if (!d3 && dk != 0) continue;
                        double w = d3 ? (dk == 0 ? 4.0 / 6.0 : 1.0 / 6.0) : 1.0;
                        double dxdy = (F(Y, i + 1, j, k + dk) - F(Y, i + 1, j - 1, k + dk))
                                    - (F(Y, i, j, k + dk) - F(Y, i, j - 1, k + dk));
                        axy += w * dxdy;
                    }
                    v += -rxy / 6.0 * axy;
                    /* A_xz Ez = -(t^2/(6 dz dx)) Dz Dx (1 + Dyy/6) Ez: Ez (i,j,k+1/2) -> Ex */
                    if (d3) {
                        double axz = 0.0;
                        for (int dj = -1; dj <= 1; dj++) {
                            double w = dj == 0 ? 4.0 / 6.0 : 1.0 / 6.0;
                            double dzdx = (F(Z, i + 1, j + dj, k) - F(Z, i + 1, j + dj, k - 1))
                                        - (F(Z, i, j + dj, k) - F(Z, i, j + dj, k - 1));
                            axz += w * dzdx;
                        }
                        v += -rzx / 6.0 * axz;
                    }
                    y[0][o] = v;
                }
                if (mask & 2) {
                    /* A_yy Ey: ((rz-1)/6) Dzz + ((rx-1)/6) Dxx + ((rz+rx-1)/36) Dzzxx */
                    double v = (rx - 1.0) / 6.0 * DXX(Y, i, j, k);
                    if (d3) v += (rz - 1.0) / 6.0 * DZZ(Y, i, j, k)
                               + (rz + rx - 1.0) / 36.0 * (DZZ(Y, i + 1, j, k) - 2.0 * DZZ(Y, i, j, k) + DZZ(Y, i - 1, j, k));
                    /* A_yx Ex: Ex (i+1/2,j,k) -> Ey (i,j+1/2,k), times alpha_z */
                    double ayx = 0.0;
                    for (int dk = -1; dk <= 1; dk++) {
                        if (!d3 && dk != 0) continue;
                        double w = d3 ? (dk == 0 ? 4.0 / 6.0 : 1.0 / 6.0) : 1.0;
                        double dydx = (F(X, i, j + 1, k + dk) - F(X, i - 1, j + 1, k + dk))
                                    - (F(X, i, j, k + dk) - F(X, i - 1, j, k + dk));
                        ayx += w * dydx;
                    }
                    v += -rxy / 6.0 * ayx;
                    /* A_yz Ez: Ez (i,j,k+1/2) -> Ey (i,j+1/2,k), times alpha_x */
                    if (d3) {
                        double ayz = 0.0;
                        for (int di = -1; di <= 1; di++) {
                            double w = di == 0 ? 4.0 / 6.0 : 1.0 / 6.0;
                            double dydz = (F(Z, i + di, j + 1, k) - F(Z, i + di, j + 1, k - 1))
                                        - (F(Z, i + di, j, k) - F(Z, i + di, j, k - 1));
                            ayz += w * dydz;
                        }
                        v += -ryz / 6.0 * ayz;
                    }
                    y[1][o] = v;
                }
                if (mask & 4) {
                    /* A_zz Ez: ((rx-1)/6) Dxx + ((ry-1)/6) Dyy + ((rx+ry-1)/36) Dxxyy */
                    double v = (rx - 1.0) / 6.0 * DXX(Z, i, j, k) + (ry - 1.0) / 6.0 * DYY(Z, i, j, k)
                             + (rx + ry - 1.0) / 36.0 * (DXX(Z, i, j + 1, k) - 2.0 * DXX(Z, i, j, k) + DXX(Z, i, j - 1, k));
                    if (d3) {
                        /* A_zx Ex: Ex (i+1/2,j,k) -> Ez (i,j,k+1/2), times alpha_y */
                        double azx = 0.0, azy = 0.0;
                        for (int dj = -1; dj <= 1; dj++) {
                            double w = dj == 0 ? 4.0 / 6.0 : 1.0 / 6.0;
                            double dzdx = (F(X, i, j + dj, k + 1) - F(X, i - 1, j + dj, k + 1))
                                        - (F(X, i, j + dj, k) - F(X, i - 1, j + dj, k));
                            azx += w * dzdx;
                        }
                        /* A_zy Ey: Ey (i,j+1/2,k) -> Ez (i,j,k+1/2), times alpha_x */
                        for (int di = -1; di <= 1; di++) {
                            double w = di == 0 ? 4.0 / 6.0 : 1.0 / 6.0;
                            double dzdy = (F(Y, i + di, j, k + 1) - F(Y, i + di, j - 1, k + 1))
                                        - (F(Y, i + di, j, k) - F(Y, i + di, j - 1, k));
                            azy += w * dzdy;
                        }
                        v += -rzx / 6.0 * azx - ryz / 6.0 * azy;
                    }
                    y[2][o] = v;
                }
#undef F
#undef DXX
#undef DYY
#undef DZZ
            }
}

/* component mask of decoupled block b */
static int block_mask(const ora_cfg *c, int b)
{
    if (c->ndim == 3) return b == 0 ? 7 : 0;
    if (b == 0) return (c->blocks & 1) ? 3 : 0;
    return (c->blocks & 2) ? 4 : 0;
}

static double norm2_mask(const ora_cfg *c, double *const a[3], double *const b[3], int mask)
{
    long n = ncell(c);
    double s = 0.0;
    for (int q = 0; q < 3; q++) {
        if (!(mask & (1 << q))) continue;
        for (long o = 0; o < n; o++) {
            double d = b ? a[q][o] - b[q][o] : a[q][o];
            s += d * d;
        }
    }
    return sqrt(s);
}

/* ------------------------------------------------------------------------ */
/* Upper end of the spectrum of A on block b (its lower end is 0): the       */
/* largest eigenvalue of the Fourier symbol of A over the Brillouin zone.    */
/* With s_i = sin^2(k_i d_i/2) the 2D TM symbol is                           */
/*   (2/3)(1-rx) sx + (2/3)(1-ry) sy - (4/9)(1-rx-ry) sx sy,                 */
/* bilinear in (sx, sy), so its maximum is at a corner of [0,1]^2; the 2D TE */
/* symbol is the 2x2 matrix [[(2/3)(1-ry) sy, m], [m, (2/3)(1-rx) sx]] with  */
/* m^2 = (4/9) rx ry sx sy, whose largest eigenvalue peaks at sx = sy = 1,   */
/* where it is 2/3 for any dt.  In 3D with cubic cells the spectrum of the   */
/* coupled 3x3 symbol fills [0, 8/9] for any dt.                             */
/* ------------------------------------------------------------------------ */
static double spectrum_top(const ora_cfg *c, int blk)
{
    double rx = c->dt * c->dt / (c->dx * c->dx), ry = c->dt * c->dt / (c->dy * c->dy);
    if (c->ndim == 3) return 8.0 / 9.0;
    if (blk == 0) return 2.0 / 3.0;
    double a = 2.0 / 3.0 * (1.0 - rx), b = 2.0 / 3.0 * (1.0 - ry), d = 8.0 / 9.0 - 2.0 / 9.0 * (rx + ry);
    double m = a > b ? a : b;
    return m > d ? m : d;
}

/* ------------------------------------------------------------------------ */
/* Chebyshev semi-iteration for (1 - A) x = b on one block, an accelerated  */
/* alternative to Alg 1 (the paper leaves faster solves to future work).     */
/* 1 - A is symmetric with its spectrum in [1 - rho, 1]; theta and delta are */
/* the centre and half width of that interval, s1 = theta/delta.  Starting   */
/* from x_0 = b, sweep k (k = 0, 1, ...) takes                               */
/*   r_k = b + A x_k - x_k                   (the residual of x_k)           */
/*   w_0 = 1/s1,  d_0 = r_0/theta                                            */
/*   w_k = 1/(2 s1 - w_(k-1)),  d_k = w_k w_(k-1) d_(k-1) + (2 w_k/delta) r_k */
/*   x_(k+1) = x_k + d_k,                                                    */
/* the three-term recurrence of the Chebyshev polynomials written with the  */
/* increments d_k.  After j sweeps x holds x_j; a tolerance stop tests       */
/* ||r_(j-1)|| <= tol ||b|| at the check points, as Alg 1 tests             */
/* ||x_j - x_(j-1)||, which is the same residual.                            */
/* ------------------------------------------------------------------------ */
static void solve_cheb_block(const ora_cfg *c, double *const b[3], double *x[3], int mask, int target,
                             int use_tol, double bn, double *tmp[3], double *d[3], int *jout, double *rout)
{
    long n = ncell(c);
    double rho = spectrum_top(c, mask == 4 ? 1 : 0);
    double theta = 1.0 - rho / 2.0, delta = rho / 2.0, s1 = theta / delta;
    double w_prev = 0.0;
    int j = 0;
    double res = 0.0;
    while (j < target) {
        ora_apply_A(c, x, tmp, mask);
        double w, cd, cr;
        if (j == 0) { w = 1.0 / s1; cd = 0.0; cr = 1.0 / theta; }
        else { w = 1.0 / (2.0 * s1 - w_prev); cd = w * w_prev; cr = 2.0 * w / delta; }
        w_prev = w;
        double s = 0.0;
        for (int q = 0; q < 3; q++) {
            if (!(mask & (1 << q))) continue;
            for (long o = 0; o < n; o++) {
                double r = b[q][o] + tmp[q][o] - x[q][o];
                s += r * r;
                d[q][o] = cd * d[q][o] + cr * r;
                x[q][o] += d[q][o];
            }
        }
        res = sqrt(s);
        j++;
        if (use_tol) {
            int g = c->check_every > 0 ? c->check_every : 1;
            if ((j % g == 0 || j == target) && res <= c->tol * bn) break;
        }
    }
    *jout = j;
    *rout = res;
}

/* ------------------------------------------------------------------------ */
/* Alg 1: x_(0) = b; x_(j+1) = b + A x_(j).  Per decoupled block: a fixed   */
/* count (tol == 0 or replay given), or stop after sweep j+1 when it is a   */
/* check point and ||x_(j+1) - x_(j)|| <= tol ||b||, or at m_max.  When     */
/* ||b|| = 0 the block takes 0 sweeps.  On return x holds the solution.     */
/* ------------------------------------------------------------------------ */
void ora_solve(const ora_cfg *c, double *const b[3], double *x[3], const int *replay, ora_stats *st)
{
    long n = ncell(c);
    double *nx_[3], *tmp[3];
    for (int q = 0; q < 3; q++) {
        nx_[q] = (double *)malloc(sizeof(double) * n);
        tmp[q] = (double *)malloc(sizeof(double) * n);
        memcpy(x[q], b[q], sizeof(double) * n);
    }
    int nb = c->ndim == 3 ? 1 : 2;
    for (int blk = 0; blk < 2; blk++) {
        st->sweeps[blk] = 0; st->resid[blk] = 0.0; st->rhs[blk] = 0.0; st->nonconverged[blk] = 0;
    }
    for (int blk = 0; blk < nb; blk++) {
        int mask = block_mask(c, blk);
        if (!mask) continue;
        double bn = norm2_mask(c, b, NULL, mask);
        st->rhs[blk] = bn;
        int target = replay ? replay[blk] : c->sweeps;
        if (c->lumped) target = 0;           /* A = 0: dE = dE' */
        if (!replay && c->tol > 0.0 && bn == 0.0) target = 0;
        int j = 0;
        double res = 0.0;
        if (c->solver == 1) {
            for (int q = 0; q < 3; q++)
                if (mask & (1 << q)) memset(nx_[q], 0, sizeof(double) * n);
            solve_cheb_block(c, b, x, mask, target, !replay && c->tol > 0.0, bn, tmp, nx_, &j, &res);
            target = 0;   /* done: skip the Alg 1 loop */
        }
        while (j < target) {
            ora_apply_A(c, x, tmp, mask);
            for (int q = 0; q < 3; q++) {
                if (!(mask & (1 << q))) continue;
                for (long o = 0; o < n; o++) nx_[q][o] = b[q][o] + tmp[q][o];
            }
            res = norm2_mask(c, nx_, x, mask);
            for (int q = 0; q < 3; q++)
                if (mask & (1 << q)) memcpy(x[q], nx_[q], sizeof(double) * n);
            j++;
            if (!replay && c->tol > 0.0) {
                int g = c->check_every > 0 ? c->check_every : 1;
                if ((j % g == 0 || j == target) && res <= c->tol * bn) break;
            }
        }
        st->sweeps[blk] = j;
        st->resid[blk] = res;
        if (!replay && c->tol > 0.0 && j > 0 && res > c->tol * bn) st->nonconverged[blk] = 1;
    }
    for (int q = 0; q < 3; q++) { free(nx_[q]); free(tmp[q]); }
}

/* ------------------------------------------------------------------------ */
/* One time step (Sec. 2.2.1): B update, dE', solve, E += dE.               */
/* J0 may be NULL; the current at n+1/2 is env * J0, filtered p times.       */
/* Returns 0, or -1 when a residual or field is not finite.                 */
/* ------------------------------------------------------------------------ */
int ora_step(const ora_cfg *c, double *E[3], double *B[3], double *const J0[3], double env,
             const int *replay, ora_stats *st)
{
    long n = ncell(c);
    double *dEp[3], *dE[3], *Jf[3] = {NULL, NULL, NULL};
    for (int q = 0; q < 3; q++) {
        dEp[q] = (double *)calloc(n, sizeof(double));
        dE[q] = (double *)calloc(n, sizeof(double));
    }
    ora_faraday(c, E, B);
    if (J0) {
        for (int q = 0; q < 3; q++) {
            Jf[q] = (double *)malloc(sizeof(double) * n);
            ora_filter(c, J0[q], Jf[q]);
        }
    }
    ora_rhs(c, B, J0 ? Jf : NULL, env, dEp);
    /* components outside the active 2D blocks stay untouched */
    if (c->ndim == 2) {
        if (!(c->blocks & 1)) { memset(dEp[0], 0, sizeof(double) * n); memset(dEp[1], 0, sizeof(double) * n); }
        if (!(c->blocks & 2)) memset(dEp[2], 0, sizeof(double) * n);
    }
    ora_solve(c, dEp, dE, replay, st);
    int bad = 0;
    for (int q = 0; q < 3; q++)
        for (long o = 0; o < n; o++) {
            E[q][o] += dE[q][o];
            if (!isfinite(E[q][o])) bad = 1;
        }
    for (int b = 0; b < 2; b++)
        if (!isfinite(st->resid[b]) || !isfinite(st->rhs[b])) bad = 1;
    for (int q = 0; q < 3; q++) { free(dEp[q]); free(dE[q]); if (Jf[q]) free(Jf[q]); }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of one step.  The forward step is linear in (E, B, J0):          */
/*   B+ = B - t K E,  E+ = E + P (t K^T Lambda B+ - 4 pi dt env F J0),      */
/* with K the E->B curl of the Faraday equations, K^T the B->E curl of the  */
/* auxiliary equations (transposes of each other on a periodic grid),       */
/* P = sum_{j<=m} A^j (Alg 1) and F the filter.  A (Appendix C), Lambda and */
/* F are symmetric, so the transposed step is                               */
/*   v = P Ebar;  Bbar += t Lambda K v;  Ebar -= t K^T Bbar;                */
/*   J0bar += env (-4 pi dt) F v.                                           */
/* `sweeps` are the per-block counts the forward step used.                 */
/* ------------------------------------------------------------------------ */
void ora_adjoint_step(const ora_cfg *c, double *Ebar[3], double *Bbar[3], double *J0bar[3],
                      double env, const int *sweeps)
{
    long n = ncell(c);
    double *v[3], *kv[3], *tmp[3];
    for (int q = 0; q < 3; q++) {
        v[q] = (double *)calloc(n, sizeof(double));
        kv[q] = (double *)calloc(n, sizeof(double));
        tmp[q] = (double *)calloc(n, sizeof(double));
    }
    ora_stats st;
    double *eb[3];
    for (int q = 0; q < 3; q++) eb[q] = Ebar[q];
    if (c->ndim == 2) {
        /* inactive blocks carry no adjoint either */
        if (!(c->blocks & 1)) { memset(Ebar[0], 0, sizeof(double) * n); memset(Ebar[1], 0, sizeof(double) * n); }
        if (!(c->blocks & 2)) memset(Ebar[2], 0, sizeof(double) * n);
    }
    ora_solve(c, eb, v, sweeps, &st);
    /* K v: the Faraday curl applied to v (sign +): kv = -(B update of zero B) */
    ora_faraday(c, v, kv);           /* kv = 0 - t K v */
    /* Lambda (K v): alpha_x on x, alpha_y on y, alpha_z on z, at B positions */
    #pragma omp parallel for collapse(2)
    for (long k = 0; k < c->nz; k++)
        for (long j = 0; j < c->ny; j++)
            for (long i = 0; i < c->nx; i++) {
                long o = IDX(c, i, j, k);
                int L = c->lumped;
                double ax = avg3(kv[0][IDX(c, i - 1, j, k)], kv[0][o], kv[0][IDX(c, i + 1, j, k)], L);
                double ay = avg3(kv[1][IDX(c, i, j - 1, k)], kv[1][o], kv[1][IDX(c, i, j + 1, k)], L);
                double az = c->ndim == 3 ? avg3(kv[2][IDX(c, i, j, k - 1)], kv[2][o], kv[2][IDX(c, i, j, k + 1)], L)
                                         : kv[2][o];
                /* kv holds -t K v, so B-bar += t Lambda K v is a subtraction */
                tmp[0][o] = ax; tmp[1][o] = ay; tmp[2][o] = az;
            }
    for (int q = 0; q < 3; q++)
        for (long o = 0; o < n; o++) Bbar[q][o] -= tmp[q][o];
    /* E-bar -= t K^T B-bar: K^T is the curl of the auxiliary equations with
       Lambda = 1, i.e. ora_rhs of the lumped scheme without a source */
    ora_cfg cl = *c;
    cl.lumped = 1;
    ora_rhs(&cl, Bbar, NULL, 0.0, tmp);   /* tmp = t K^T Bbar */
    for (int q = 0; q < 3; q++)
        for (long o = 0; o < n; o++) Ebar[q][o] -= tmp[q][o];
    if (c->ndim == 2) {
        if (!(c->blocks & 1)) { memset(Ebar[0], 0, sizeof(double) * n); memset(Ebar[1], 0, sizeof(double) * n); }
        if (!(c->blocks & 2)) memset(Ebar[2], 0, sizeof(double) * n);
    }
    if (J0bar) {
        double s = -c->four_pi * c->dt * env;
        for (int q = 0; q < 3; q++) {
            ora_filter(c, v[q], tmp[q]);
            for (long o = 0; o < n; o++) J0bar[q][o] += s * tmp[q][o];
        }
    }
    for (int q = 0; q < 3; q++) { free(v[q]); free(kv[q]); free(tmp[q]); }
}

#ifdef _OPENMP
#include <omp.h>
#endif
int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads the next parallel regions use (n >= 1); the CPU-baseline timing
   runs the oracle on all host cores and on one. */
void ora_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * Particle coupling in 2D with three velocity components.  The paper runs
 * the field solver inside a particle-in-cell code and keeps that code's
 * force interpolation, current deposition and particle push (Sec. 2: only
 * Faraday's and Ampere's equations change); Gauss's law for E then holds
 * because the deposition conserves charge (Sec. 2, Appendix A).  The
 * particle side is written here from the published methods it names:
 *   push ........ the relativistic Boris scheme (Boris 1970; the push of
 *                 the paper's experiments, Sec. 5): half electric kick,
 *                 magnetic rotation, half electric kick, then the move
 *   shapes ...... first-order B-spline (linear weighting) at each field
 *                 component's staggered position, the lowest order of the
 *                 paper's Table 1, the same shape for interpolation and
 *                 deposition
 *   deposition .. Esirkepov's charge-conserving density decomposition
 *                 (Esirkepov 2001) in its 2D form with an out-of-plane
 *                 current, so rho^{n+1} - rho^n + dt D.J^{n+1/2} = 0 holds
 *                 exactly on the nodes
 * Time levels: positions at n, momenta u = gamma v at n - 1/2 (c = 1); the
 * force uses E^n and B^n = (B^{n-1/2} + B^{n+1/2})/2 = B^{n-1/2} - (dt/2)
 * curl E^n; the move gives positions at n + 1 and the current J^{n+1/2}
 * that the field step then uses (env = 1).  Positions are physical
 * coordinates with node (i, j) at (i dx, j dy), kept in [0, L) by periodic
 * wrapping.  rho and J are densities per cell area: a macro-particle of
 * charge q and weight w carries charge q w.
 * ------------------------------------------------------------------------ */

/* linear B-spline */
static double shape1(double d)
{
    d = fabs(d);
    return d < 1.0 ? 1.0 - d : 0.0;
}

/* F at (x, y) interpolated with the linear shape; F sits at (i + ox, j + oy) cells */
static double gather1(const ora_cfg *c, const double *F, double x, double y, double ox, double oy)
{
    const double xi = x / c->dx - ox, eta = y / c->dy - oy;
    const long i0 = (long)floor(xi), j0 = (long)floor(eta);
    double v = 0.0;
    for (int b = 0; b < 2; b++)
        for (int a = 0; a < 2; a++) {
            const double wgt = shape1(xi - (double)(i0 + a)) * shape1(eta - (double)(j0 + b));
            v += wgt * F[IDX(c, i0 + a, j0 + b, 0)];
        }
    return v;
}

static double wrap_pos(double x, double L)
{
    if (x >= L) return x - L;
    if (x < 0.0) return x + L;
    return x;
}

/* push np particles of charge q, mass m and weight w through one step and
   add their current J^{n+1/2} into J; returns 1 if a particle would cross
   more than one cell (the deposition stencil assumes |v| dt < cell), else 0 */
int ora_pic_push_deposit(const ora_cfg *c, double *const E[3], double *const B[3], long np, double q, double m,
                         double w, double *x, double *y, double *ux, double *uy, double *uz, double *const J[3])
{
    const long n = ncell(c);
    const double dt = c->dt;
    const double Lx = c->nx * c->dx, Ly = c->ny * c->dy;
    /* B^n: half a Faraday step from B^{n-1/2} with E^n */
    double *Bn[3];
    for (int q3 = 0; q3 < 3; q3++) {
        Bn[q3] = (double *)malloc(sizeof(double) * n);
        memcpy(Bn[q3], B[q3], sizeof(double) * n);
    }
    ora_cfg half = *c;
    half.dt = 0.5 * dt;
    ora_faraday(&half, E, Bn);
    const double h = q * dt / (2.0 * m);
    const double cx = -q * w / (c->dy * dt), cy = -q * w / (c->dx * dt), cz = q * w / (c->dx * c->dy);
    int bad = 0;
    for (long p = 0; p < np; p++) {
        const double x0 = x[p], y0 = y[p];
        /* field at the particle (staggered positions of Sec. 2) */
        const double ex = gather1(c, E[0], x0, y0, 0.5, 0.0);
        const double ey = gather1(c, E[1], x0, y0, 0.0, 0.5);
        const double ez = gather1(c, E[2], x0, y0, 0.0, 0.0);
        const double bx = gather1(c, Bn[0], x0, y0, 0.0, 0.5);
        const double by = gather1(c, Bn[1], x0, y0, 0.5, 0.0);
        const double bz = gather1(c, Bn[2], x0, y0, 0.5, 0.5);
        /* Boris: u- = u + h E; rotate about B by the angle of t = h B / gamma-;
           u+ = u- + (u- + u- x t) x s, s = 2 t / (1 + t.t); u = u+ + h E */
        const double umx = ux[p] + h * ex, umy = uy[p] + h * ey, umz = uz[p] + h * ez;
        const double gm = sqrt(1.0 + umx * umx + umy * umy + umz * umz);
        const double tx = h * bx / gm, ty = h * by / gm, tz = h * bz / gm;
        const double upx = umx + (umy * tz - umz * ty);
        const double upy = umy + (umz * tx - umx * tz);
        const double upz = umz + (umx * ty - umy * tx);
        const double f = 2.0 / (1.0 + tx * tx + ty * ty + tz * tz);
        const double sx = f * tx, sy = f * ty, sz = f * tz;
        const double uplx = umx + (upy * sz - upz * sy);
        const double uply = umy + (upz * sx - upx * sz);
        const double uplz = umz + (upx * sy - upy * sx);
        const double nux = uplx + h * ex, nuy = uply + h * ey, nuz = uplz + h * ez;
        const double g = sqrt(1.0 + nux * nux + nuy * nuy + nuz * nuz);
        const double x1 = x0 + dt * nux / g, y1 = y0 + dt * nuy / g;
        /* Esirkepov: local 4 x 4 node window starting one node left of the
           particle's start cell */
        const double xi0 = x0 / c->dx, eta0 = y0 / c->dy, xi1 = x1 / c->dx, eta1 = y1 / c->dy;
        if (fabs(xi1 - xi0) >= 1.0 || fabs(eta1 - eta0) >= 1.0) bad = 1;
        const long i0 = (long)floor(xi0) - 1, j0 = (long)floor(eta0) - 1;
        double sx0[4], sx1[4], sy0[4], sy1[4];
        for (int k = 0; k < 4; k++) {
            sx0[k] = shape1(xi0 - (double)(i0 + k));
            sx1[k] = shape1(xi1 - (double)(i0 + k));
            sy0[k] = shape1(eta0 - (double)(j0 + k));
            sy1[k] = shape1(eta1 - (double)(j0 + k));
        }
        const double vz = nuz / g;
        for (int l = 0; l < 4; l++) {
            double run = 0.0;   /* sum over k' <= k of W_x(k', l) */
            for (int k = 0; k < 4; k++) {
                const double wx = 0.5 * (sx1[k] - sx0[k]) * (sy0[l] + sy1[l]);
                run += wx;
                if (k < 3) J[0][IDX(c, i0 + k, j0 + l, 0)] += cx * run;
            }
        }
        for (int k = 0; k < 4; k++) {
            double run = 0.0;   /* sum over l' <= l of W_y(k, l') */
            for (int l = 0; l < 4; l++) {
                const double wy = 0.5 * (sy1[l] - sy0[l]) * (sx0[k] + sx1[k]);
                run += wy;
                if (l < 3) J[1][IDX(c, i0 + k, j0 + l, 0)] += cy * run;
            }
        }
        for (int l = 0; l < 4; l++)
            for (int k = 0; k < 4; k++) {
                const double wz = (2.0 * sx0[k] * sy0[l] + sx1[k] * sy0[l] + sx0[k] * sy1[l] + 2.0 * sx1[k] * sy1[l]) / 6.0;
                J[2][IDX(c, i0 + k, j0 + l, 0)] += cz * vz * wz;
            }
        x[p] = wrap_pos(x1, Lx);
        y[p] = wrap_pos(y1, Ly);
        ux[p] = nux;
        uy[p] = nuy;
        uz[p] = nuz;
    }
    for (int q3 = 0; q3 < 3; q3++) free(Bn[q3]);
    return bad;
}

/* rho at the nodes (i, j) += q w / (dx dy) S(x/dx - i) S(y/dy - j) */
void ora_pic_deposit_charge(const ora_cfg *c, long np, double q, double w, const double *x, const double *y,
                            double *rho)
{
    const double cq = q * w / (c->dx * c->dy);
    for (long p = 0; p < np; p++) {
        const double xi = x[p] / c->dx, eta = y[p] / c->dy;
        const long i0 = (long)floor(xi), j0 = (long)floor(eta);
        for (int b = 0; b < 2; b++)
            for (int a = 0; a < 2; a++)
                rho[IDX(c, i0 + a, j0 + b, 0)] +=
                    cq * shape1(xi - (double)(i0 + a)) * shape1(eta - (double)(j0 + b));
    }
}
