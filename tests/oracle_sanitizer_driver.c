/* Drives the oracle under AddressSanitizer and UndefinedBehaviorSanitizer (built
 * by tests/test_oracle_sanitizer.py with gcc): every PDE in 2-D and 3-D, the
 * emulated formats, storage rounding, the paper semantics, the CK predictor, the
 * sampled-cell step, receivers and the adjoint step on small grids.  Exits 0
 * when every call succeeds and the states stay finite; the sanitizers abort on
 * any memory or undefined-behaviour error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "aderdg_oracle.h"

static int finite_state(const or_solver *s)
{
    size_t n = (size_t)s->ncell * s->V * s->S;
    double *Q = malloc(sizeof(double) * n);
    or_get_state(s, Q);
    int ok = 1;
    for (size_t i = 0; i < n; i++) ok &= isfinite(Q[i]);
    free(Q);
    return ok;
}

static int run(int pde, int dim, int order, const double *params, int p, int storage, int sem, int pred)
{
    or_config c;
    memset(&c, 0, sizeof(c));
    c.dim = dim;
    c.order = order;
    for (int i = 0; i < 3; i++) { c.cells[i] = i < dim ? 3 + i : 1; c.lo[i] = 0.0; c.hi[i] = (3 + i) * 0.25; }
    c.pde = pde;
    for (int i = 0; i < 8; i++) c.params[i] = params[i];
    c.prec[0] = p; c.prec[1] = p; c.prec[2] = sem ? p : OR_FP64;
    c.storage = storage;
    c.semantics = sem;
    c.prec_picard = -1;
    c.predictor = pred;
    or_solver *s = or_create(&c);
    if (!s) { fprintf(stderr, "create failed pde %d dim %d\n", pde, dim); return 1; }
    size_t n = (size_t)s->ncell * s->V * s->S;
    double *Q = malloc(sizeof(double) * n);
    for (size_t i = 0; i < n; i++) Q[i] = 0.01 * sin(0.37 * (double)i);
    if (pde == OR_EULER)
        for (int64_t e = 0; e < s->ncell; e++)
            for (int k = 0; k < s->S; k++) {
                Q[(e * s->V + 0) * s->S + k] += 1.0;         /* density */
                Q[(e * s->V + s->V - 1) * s->S + k] += 2.5;  /* energy */
            }
    if (pde == OR_SWE)
        for (int64_t e = 0; e < s->ncell; e++)
            for (int k = 0; k < s->S; k++) Q[(e * s->V + 0) * s->S + k] += 2.0;
    or_set_state(s, Q);
    if (pde == OR_ACOUSTIC && !sem && pred == OR_PICARD) {
        double *cm = malloc(sizeof(double) * s->ncell);
        for (int64_t e = 0; e < s->ncell; e++) cm[e] = 1.0 + 0.1 * (double)(e % 3);
        or_set_material(s, cm);
        free(cm);
        double xs[3] = {0.3, 0.4, 0.2};
        or_set_source(s, xs, 5.0, 0.2, 1.0);
    }
    double dt = or_max_dt(s, 0.4);
    int rc = 0;
    for (int k = 0; k < 2; k++) rc |= or_step(s, k * dt, dt);
    int64_t ids[2] = {0, s->ncell - 1};
    double *out = malloc(sizeof(double) * 2 * s->V * s->S);
    rc |= or_step_cells(s, 2 * dt, dt, 2, ids, out);
    double pts[3] = {0.31, 0.52, 0.1}, val;
    rc |= or_sample_points(s, 1, pts, 0, &val);
    if (pde == OR_ACOUSTIC && !sem && pred == OR_PICARD && storage == OR_FP64 && (p == OR_FP64)) {
        double *lam = malloc(sizeof(double) * n), *mu = malloc(sizeof(double) * n);
        double *g = calloc((size_t)s->ncell, sizeof(double));
        for (size_t i = 0; i < n; i++) lam[i] = cos(0.11 * (double)i);
        rc |= or_adjoint_step(s, Q, 0.0, dt, lam, mu, g);
        free(lam); free(mu); free(g);
    }
    int ok = finite_state(s) && rc == 0;
    free(out);
    free(Q);
    or_destroy(s);
    if (!ok) fprintf(stderr, "failed pde %d dim %d order %d p %d storage %d sem %d pred %d\n", pde, dim, order, p,
                     storage, sem, pred);
    return ok ? 0 : 1;
}

int main(void)
{
    const double ac[8] = {1.0, 2.25}, el[8] = {2.7, 32.4, 32.4}, eu[8] = {1.4}, sw[8] = {9.81};
    int fail = 0;
    for (int dim = 2; dim <= 3; dim++)
        for (int p = OR_FP64; p <= OR_FP16; p++) {
            fail |= run(OR_ACOUSTIC, dim, 2, ac, p, OR_FP64, OR_SEM_BUILD, OR_PICARD);
            fail |= run(OR_ELASTIC, dim, 2, el, p, p, OR_SEM_BUILD, OR_PICARD);
            fail |= run(OR_EULER, dim, 2, eu, p, OR_FP64, OR_SEM_BUILD, OR_PICARD);
            fail |= run(OR_ACOUSTIC, dim, 2, ac, p, p, OR_SEM_PAPER, OR_PICARD);
            fail |= run(OR_ELASTIC, dim, 3, el, p, OR_FP64, OR_SEM_BUILD, OR_CK);
        }
    for (int p = OR_FP64; p <= OR_FP16; p++) {
        fail |= run(OR_SWE, 2, 3, sw, p, OR_FP64, OR_SEM_BUILD, OR_PICARD);
        fail |= run(OR_SWE, 2, 2, sw, p, p, OR_SEM_PAPER, OR_PICARD);
        fail |= run(OR_EULER, 2, 1, eu, p, p, OR_SEM_PAPER, OR_PICARD);
    }
    double xi[8], w[8], D[64], F0[8], F1[8], K1[64], At[64], Kx[64], L0[8], L1[8];
    for (int n = 1; n <= 8; n++) fail |= or_basis(n, xi, w, D, F0, F1, K1, At, Kx, L0, L1) != 0;
    printf(fail ? "FAILED\n" : "OK\n");
    return fail;
}
