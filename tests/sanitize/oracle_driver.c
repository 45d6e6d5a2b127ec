/*
 * Runs every entry point of the FP64 oracle once on small periodic grids,
 * built together with the oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (the test that builds it passes the flags):
 * any out-of-bounds access, leak, use after free, signed overflow or bad
 * shift ends the run with a report and a non-zero status.  Grid sizes are
 * odd and unequal so that every wrap of the periodic index is taken.
 */
#include "../../oracle/mx_oracle.c"

#include <stdio.h>

static unsigned long long rng_state = 0x9e3779b97f4a7c15ull;

static double urand(void) /* splitmix64 -> [-1, 1) */
{
    unsigned long long z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static double *field(long n, double scale)
{
    double *f = (double *)malloc((size_t)n * sizeof(double));
    for (long i = 0; i < n; i++) f[i] = scale * urand();
    return f;
}

static int run(const ora_cfg *c, int nsteps)
{
    const long n = c->nx * c->ny * c->nz;
    double *E[3], *B[3], *J0[3], *Eb[3], *Bb[3], *Jb[3];
    for (int q = 0; q < 3; q++) {
        E[q] = field(n, 1.0);
        B[q] = field(n, 1.0);
        J0[q] = field(n, 0.1);
        Eb[q] = field(n, 1.0);
        Bb[q] = field(n, 1.0);
        Jb[q] = field(n, 0.0);
    }
    int rc = 0;
    ora_stats st;
    for (int s = 0; s < nsteps && rc == 0; s++) rc = ora_step(c, E, B, J0, 0.5 + 0.1 * s, NULL, &st);
    const int sw[2] = {st.sweeps[0], st.sweeps[1]};
    ora_adjoint_step(c, Eb, Bb, Jb, 0.7, sw);
    if (c->ndim == 2) {
        const long np = 97;
        double *x = field(np, 0.0), *y = field(np, 0.0), *ux = field(np, 2.0), *uy = field(np, 2.0),
               *uz = field(np, 2.0), *rho = field(n, 0.0), *J[3];
        for (long p = 0; p < np; p++) {
            /* positions anywhere in the box, some on its edges */
            x[p] = (p % 7 == 0) ? 0.0 : (0.5 + 0.5 * urand()) * c->nx * c->dx;
            y[p] = (p % 11 == 0) ? (c->ny - 1e-12) * c->dy : (0.5 + 0.5 * urand()) * c->ny * c->dy;
        }
        for (int q = 0; q < 3; q++) J[q] = field(n, 0.0);
        ora_pic_push_deposit(c, E, B, np, -1.0, 1.0, 0.01, x, y, ux, uy, uz, J);
        ora_pic_deposit_charge(c, np, -1.0, 0.01, x, y, rho);
        for (int q = 0; q < 3; q++) free(J[q]);
        free(x); free(y); free(ux); free(uy); free(uz); free(rho);
    }
    for (int q = 0; q < 3; q++) {
        free(E[q]); free(B[q]); free(J0[q]); free(Eb[q]); free(Bb[q]); free(Jb[q]);
    }
    return rc;
}

int main(void)
{
    ora_set_num_threads(2);
    const double fp = 4.0 * 3.14159265358979323846;
    /* 2D TE+TM: fixed sweeps, tolerance stop, Chebyshev, lumped */
    ora_cfg c2 = {2, 13, 9, 1, 1.0, 0.8, 1.0, 0.3, 3, 6, 0.0, 1, 3, 0, fp, 0};
    int rc = run(&c2, 3);
    c2.tol = 1e-10; c2.sweeps = 60; c2.check_every = 2;
    rc |= run(&c2, 2);
    c2.tol = 0.0; c2.sweeps = 8; c2.solver = 1;
    rc |= run(&c2, 2);
    c2.solver = 0; c2.lumped = 1; c2.filter_passes = 0;
    rc |= run(&c2, 2);
    /* 2D single block each */
    ora_cfg c2te = {2, 11, 7, 1, 1.0, 1.0, 1.0, 0.35, 1, 5, 0.0, 1, 1, 0, fp, 0};
    rc |= run(&c2te, 2);
    c2te.blocks = 2;
    rc |= run(&c2te, 2);
    /* 3D: Alg 1, tolerance, Chebyshev on a cube */
    ora_cfg c3 = {3, 7, 5, 9, 1.0, 0.9, 1.1, 0.25, 3, 4, 0.0, 1, 2, 0, fp, 0};
    rc |= run(&c3, 2);
    c3.tol = 1e-9; c3.sweeps = 40;
    rc |= run(&c3, 1);
    ora_cfg c3c = {3, 6, 6, 6, 1.0, 1.0, 1.0, 0.25, 3, 6, 0.0, 1, 1, 0, fp, 1};
    rc |= run(&c3c, 1);
    printf("oracle sanitizer run: %s\n", rc == 0 ? "clean" : "a step reported a non-finite value");
    return rc != 0;
}
