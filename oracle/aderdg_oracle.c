/*
 * Plain FP64 CPU oracle of the ADER-DG time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the GPU library under paper_2504_06889_amd/, and the GPU
 * library never loads it.
 *
 * Method: arXiv 2504.06889, Sec. 3 ("The ADER-DG method").
 *   - Nodal tensor-product Lagrange basis on Gauss-Legendre support points
 *     (eq. piecewise_solution, and the text after eq. discreteFlux).
 *   - Predictor: the cell-local space-time DG system of eq. Picard, solved by
 *     fixed-point (Picard) iteration; the nodal flux is F(q) at each node.
 *   - Corrector: the one-step weak form eq. weak_form_volume_surface with its
 *     volume integral and the surface integral of the numerical flux.
 *   - Numerical flux: Rusanov (eq. rusanov_flux); for shallow water the
 *     well-balanced variant of eq. swe_custom_riemann.
 *   - Time step: the CFL rule eq. CFL_condition.
 *   - Algorithm 1 fixes the order: predictor, face projection and volume
 *     integral per cell, then Riemann solve and face integral per face.
 *
 * Everything is written out in the plainest form: loops over cells, nodes and
 * variables, one contraction at a time, FP64 throughout.  The optional
 * "emulated precision" mode rounds the inputs of the contractions named in
 * the header to a lower format (round-to-nearest-even) and accumulates them
 * in FP32; everything else stays FP64.  It predicts the error level of the
 * GPU mixed-precision path; it is not meant to reproduce its bits.
 *
 * Readings of points the paper leaves open (all documented in the header):
 *   Picard iterations I = N+1 from the initial guess q = Q^n at every time
 *   node; one Riemann solve per face on the time-averaged face states and
 *   fluxes; Rusanov speed taken pointwise per face node over both sides.
 */
#include "aderdg_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXN OR_MAXN
#define MAXV OR_MAXV
#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Reduced-precision rounding (format table of Sec. 1: significant bits).    */
/* ------------------------------------------------------------------------ */

/* Round a float to a binary format with `sig` significant bits (implicit bit
 * included), smallest normal exponent `emin` (value 2^emin), largest finite
 * value `maxv`; round-to-nearest-even, gradual underflow, overflow -> inf.   */
static float round_format(float f, int sig, int emin, double maxv)
{
    if (!isfinite(f) || f == 0.0f) return f;
    double a = fabs((double)f);
    double q; /* quantum (spacing of representable numbers around a) */
    if (a < ldexp(1.0, emin)) {
        q = ldexp(1.0, emin - (sig - 1));
    } else {
        int e;
        frexp(a, &e); /* a = m * 2^e with m in [0.5, 1) */
        q = ldexp(1.0, e - sig);
    }
    double r = rint(a / q) * q; /* a/q exact (power-of-two scaling); rint is RNE */
    if (r > maxv) r = INFINITY;
    return (float)copysign(r, (double)f);
}

double or_round(int p, double x)
{
    switch (p) {
    case OR_FP64: return x;
    case OR_FP32: return (double)(float)x;
    case OR_BF16: return (double)round_format((float)x, 8, -126, 3.3895313892515355e38);
    case OR_FP16: return (double)round_format((float)x, 11, -14, 65504.0);
    default: return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre nodes and the nodal Lagrange basis on [0,1].               */
/* ------------------------------------------------------------------------ */

/* Legendre polynomial P_n and its derivative at x (three-term recurrence). */
static void legendre(int n, double x, double *p, double *dp)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int k = 2; k <= n; k++) {
        double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    *p = p1;
    *dp = n * (x * p1 - p0) / (x * x - 1.0);
}

/* n Gauss-Legendre points and weights on [0,1] (ascending); sum of weights 1. */
static void gauss_legendre(int n, double *xi, double *w)
{
    for (int i = 0; i < n; i++) {
        double x = cos(PI * (i + 0.75) / (n + 0.5)); /* descending roots on [-1,1] */
        for (int it = 0; it < 100; it++) {
            double p, dp;
            legendre(n, x, &p, &dp);
            double dx = p / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double p, dp;
        legendre(n, x, &p, &dp);
        xi[i] = 0.5 * (1.0 - x);
        w[i] = 1.0 / ((1.0 - x * x) * dp * dp); /* half of the [-1,1] weight */
    }
}

/* Lagrange basis psi_j(x) on the nodes, plain product formula. */
static void lagrange_eval(int n, const double *xi, double x, double *out)
{
    for (int j = 0; j < n; j++) {
        double v = 1.0;
        for (int m = 0; m < n; m++)
            if (m != j) v *= (x - xi[m]) / (xi[j] - xi[m]);
        out[j] = v;
    }
}

/* Solve A X = B for X (n x n, row-major), Gauss-Jordan with partial pivoting. */
static void solve_dense(int n, const double *A, const double *B, double *X)
{
    double M[MAXN][2 * MAXN];
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            M[i][j] = A[i * n + j];
            M[i][n + j] = B[i * n + j];
        }
    for (int c = 0; c < n; c++) {
        int piv = c;
        for (int r = c + 1; r < n; r++)
            if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
        for (int k = 0; k < 2 * n; k++) { double t = M[c][k]; M[c][k] = M[piv][k]; M[piv][k] = t; }
        double inv = 1.0 / M[c][c];
        for (int k = 0; k < 2 * n; k++) M[c][k] *= inv;
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            double f = M[r][c];
            for (int k = 0; k < 2 * n; k++) M[r][k] -= f * M[c][k];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) X[i * n + j] = M[i][n + j];
}

int or_basis(int n, double *xi, double *w, double *D, double *F0, double *F1,
             double *K1, double *Atau, double *Kxi, double *L0, double *L1)
{
    if (n < 1 || n > MAXN) return -1;
    gauss_legendre(n, xi, w);
    /* D[i][j] = psi_j'(xi_i): barycentric form off the diagonal, and the
     * negative-sum rule on the diagonal so that D applied to a constant is 0. */
    double lam[MAXN];
    for (int j = 0; j < n; j++) {
        double pr = 1.0;
        for (int m = 0; m < n; m++)
            if (m != j) pr *= xi[j] - xi[m];
        lam[j] = 1.0 / pr;
    }
    for (int i = 0; i < n; i++) {
        double diag = 0.0;
        for (int j = 0; j < n; j++) {
            if (j == i) continue;
            D[i * n + j] = (lam[j] / lam[i]) / (xi[i] - xi[j]);
            diag -= D[i * n + j];
        }
        D[i * n + i] = diag;
    }
    lagrange_eval(n, xi, 0.0, F0);
    lagrange_eval(n, xi, 1.0, F1);
    /* Time matrix of eq. Picard on the reference interval: the first bracket,
     * K1[k][l] = psi_k(1) psi_l(1) - int psi_k' psi_l, with the integral done by
     * the (exact) Gauss rule: int psi_k' psi_l = w_l D[l][k].                  */
    double W[MAXN * MAXN];
    memset(W, 0, sizeof(W));
    for (int k = 0; k < n; k++) {
        W[k * n + k] = w[k];
        for (int l = 0; l < n; l++) K1[k * n + l] = F1[k] * F1[l] - w[l] * D[l * n + k];
    }
    /* Picard operator A_tau = K1^{-1} W: q = 1*Q - dt A_tau R (see predictor). */
    solve_dense(n, K1, W, Atau);
    /* Weak-form volume matrix (eq. weak_form_volume_surface divided by the
     * diagonal Gauss mass): Kxi[k][l] = w_l D[l][k] / w_k.  Face lifts:
     * L0 = psi(0)/w, L1 = psi(1)/w.                                           */
    for (int k = 0; k < n; k++) {
        for (int l = 0; l < n; l++) Kxi[k * n + l] = w[l] * D[l * n + k] / w[k];
        L0[k] = F0[k] / w[k];
        L1[k] = F1[k] / w[k];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* PDE systems (Sec. 5): flux, largest |eigenvalue|, non-conservative part. */
/* ------------------------------------------------------------------------ */

int or_nvars(int pde, int dim)
{
    switch (pde) {
    case OR_ACOUSTIC: return 1 + dim;
    case OR_ELASTIC: return dim * (dim + 1) / 2 + dim;
    case OR_EULER: return 2 + dim;
    case OR_SWE: return dim == 2 ? 4 : -1;
    }
    return -1;
}

/* Index of the stress component sigma_ab (a,b < d) in the elastic state. */
static int stress_index(int d, int a, int b)
{
    if (a == b) return a;
    if (a > b) { int t = a; a = b; b = t; }
    if (d == 2) return 2;                       /* sxy */
    if (a == 0 && b == 1) return 3;             /* sxy */
    if (a == 1 && b == 2) return 4;             /* syz */
    return 5;                                   /* sxz */
}

static double cell_bulk(const or_solver *s, int64_t cell)
{
    /* acoustics: K = rho c^2 with per-cell c when a material is set */
    if (s->cmat) return s->c.params[0] * s->cmat[cell] * s->cmat[cell];
    return s->c.params[1];
}

/* Physical flux F_j(q) (eq. exa_canonical_form, the conservative part). */
static void pde_flux(const or_solver *s, int64_t cell, const double *q, int j, double *F)
{
    const int d = s->d;
    const double *pr = s->c.params;
    switch (s->c.pde) {
    case OR_ACOUSTIC: { /* eq. acoustic: p_t + K div v = 0, rho v_t + grad p = 0 */
        double rho = pr[0], K = cell_bulk(s, cell);
        F[0] = K * q[1 + j];
        for (int i = 0; i < d; i++) F[1 + i] = (i == j) ? q[0] / rho : 0.0;
        break;
    }
    case OR_ELASTIC: { /* eq. equations_of_motion, written as q_t + A_j q_j = 0 */
        double rho = pr[0], lam = pr[1], mu = pr[2];
        int ns = d * (d + 1) / 2;
        const double *v = q + ns;
        for (int a = 0; a < d; a++)
            for (int b = a; b < d; b++) {
                int k = stress_index(d, a, b);
                if (a == b)
                    F[k] = -(lam + (a == j ? 2.0 * mu : 0.0)) * v[j];
                else
                    F[k] = -mu * ((b == j ? v[a] : 0.0) + (a == j ? v[b] : 0.0));
            }
        for (int i = 0; i < d; i++) F[ns + i] = -q[stress_index(d, i, j)] / rho;
        break;
    }
    case OR_EULER: { /* conserved (rho, rho v, E); energy flux v_j (E + p) */
        double g = pr[0], rho = q[0], E = q[1 + d];
        double ke = 0.0;
        for (int i = 0; i < d; i++) ke += q[1 + i] * q[1 + i];
        double p = (g - 1.0) * (E - 0.5 * ke / rho);
        double uj = q[1 + j] / rho;
        F[0] = q[1 + j];
        for (int i = 0; i < d; i++) F[1 + i] = q[1 + i] * uj + (i == j ? p : 0.0);
        F[1 + d] = uj * (E + p);
        break;
    }
    case OR_SWE: { /* conservative part (h u_j, h u u_j, h v u_j, 0) */
        double hh = q[0], uj = q[1 + j] / hh;
        F[0] = q[1 + j];
        F[1] = q[1] * uj;
        F[2] = q[2] * uj;
        F[3] = 0.0;
        break;
    }
    }
}

/* Largest |eigenvalue| of the flux Jacobian in direction j. */
static double pde_max_eig(const or_solver *s, int64_t cell, const double *q, int j)
{
    const int d = s->d;
    const double *pr = s->c.params;
    switch (s->c.pde) {
    case OR_ACOUSTIC: return sqrt(cell_bulk(s, cell) / pr[0]);
    case OR_ELASTIC: return sqrt((pr[1] + 2.0 * pr[2]) / pr[0]);
    case OR_EULER: {
        double g = pr[0], rho = q[0], E = q[1 + d], ke = 0.0;
        for (int i = 0; i < d; i++) ke += q[1 + i] * q[1 + i];
        double p = (g - 1.0) * (E - 0.5 * ke / rho);
        return fabs(q[1 + j] / rho) + sqrt(g * p / rho);
    }
    case OR_SWE: return fabs(q[1 + j] / q[0]) + sqrt(pr[0] * q[0]);
    }
    return 0.0;
}

/* Non-conservative product B_j(q) (d/dxi_j) q for shallow water (eq.
 * swe_noncons): g h d(h+b)/dxi_j in the j-momentum.  `deta` is the reference
 * derivative of eta = h + b (one contraction of eta, not of h and b apart).  */
static void swe_ncp(const or_solver *s, double h, double deta, int j, double *out)
{
    out[0] = 0.0; out[1] = 0.0; out[2] = 0.0; out[3] = 0.0;
    out[1 + j] = s->c.params[0] * h * deta;
}

/* Ricker wavelet (point-source time function). */
static double ricker(const or_solver *s, double t)
{
    double a = PI * PI * s->src_f0 * s->src_f0 * (t - s->src_t0) * (t - s->src_t0);
    return s->src_amp * (1.0 - 2.0 * a) * exp(-a);
}

/* ------------------------------------------------------------------------ */
/* Index helpers: node s = i0 + n (i1 + n i2); cell = c0 + C0 (c1 + C1 c2).  */
/* ------------------------------------------------------------------------ */

static int coord(int sn, int j, int n)
{
    for (int i = 0; i < j; i++) sn /= n;
    return sn % n;
}

static int stride_of(int j, int n)
{
    int st = 1;
    for (int i = 0; i < j; i++) st *= n;
    return st;
}

/* face node index: the node's coordinates with coordinate j removed */
static int face_of(int sn, int j, int n, int d)
{
    int f = 0, m = 1;
    for (int i = 0; i < d; i++) {
        if (i == j) continue;
        f += coord(sn, i, n) * m;
        m *= n;
    }
    return f;
}

static int64_t neighbour(const or_solver *s, int64_t cell, int j, int dir)
{
    int64_t c[3] = {0, 0, 0}, r = cell;
    for (int i = 0; i < s->d; i++) { c[i] = r % s->c.cells[i]; r /= s->c.cells[i]; }
    c[j] = (c[j] + dir + s->c.cells[j]) % s->c.cells[j];
    int64_t out = 0, m = 1;
    for (int i = 0; i < s->d; i++) { out += c[i] * m; m *= s->c.cells[i]; }
    return out;
}

/* One line contraction sum_k m[k] x[k*stride], in FP64 or emulated precision p
 * (inputs rounded to p, products and sum in FP32). */
static double contract(int n, const double *m, const double *x, int stride, int p)
{
    if (p == OR_FP64) {
        double a = 0.0;
        for (int k = 0; k < n; k++) a += m[k] * x[k * stride];
        return a;
    }
    float a = 0.0f;
    for (int k = 0; k < n; k++) {
        float mk = (float)or_round(p, m[k]);
        float xk = (float)or_round(p, x[k * stride]);
        float pk = mk * xk;
        a = a + pk;
    }
    return (double)a;
}

/* out[v][s] = sum_k M[s_j][k] X[v][s with s_j = k]  (matrix along direction j) */
static void apply_dir(const or_solver *s, const double *M, int j, const double *X, double *out,
                      int nv, int p)
{
    const int n = s->n, S = s->S, st = stride_of(j, n);
    for (int v = 0; v < nv; v++)
        for (int sn = 0; sn < S; sn++) {
            int i = coord(sn, j, n);
            const double *line = X + v * S + (sn - i * st);
            out[v * S + sn] = contract(n, M + i * n, line, st, p);
        }
}

/* ------------------------------------------------------------------------ */
/* Solver object                                                             */
/* ------------------------------------------------------------------------ */

or_solver *or_create(const or_config *cfg)
{
    if (cfg->dim < 1 || cfg->dim > 3 || cfg->order < 0 || cfg->order + 1 > MAXN) return NULL;
    int V = or_nvars(cfg->pde, cfg->dim);
    if (V <= 0 || V > MAXV) return NULL;
    if (cfg->storage < OR_FP64 || cfg->storage > OR_FP16) return NULL;
    if (cfg->semantics == OR_SEM_PAPER && (cfg->predictor != OR_PICARD || cfg->prec_picard > OR_FP16))
        return NULL; /* paper semantics: Picard predictor only */
    if (cfg->predictor != OR_PICARD &&
        (cfg->predictor != OR_CK || (cfg->pde != OR_ACOUSTIC && cfg->pde != OR_ELASTIC)))
        return NULL; /* the CK procedure needs a linear flux */
    or_solver *s = (or_solver *)calloc(1, sizeof(or_solver));
    s->c = *cfg;
    s->d = cfg->dim;
    s->n = cfg->order + 1;
    s->V = V;
    s->S = 1;
    for (int i = 0; i < s->d; i++) s->S *= s->n;
    s->F = s->S / s->n;
    s->I = cfg->picard_iters > 0 ? cfg->picard_iters : cfg->order + 1;
    s->ncell = 1;
    for (int i = 0; i < s->d; i++) s->ncell *= cfg->cells[i];
    s->h = (cfg->hi[0] - cfg->lo[0]) / cfg->cells[0];
    for (int i = 1; i < s->d; i++) {
        double hi = (cfg->hi[i] - cfg->lo[i]) / cfg->cells[i];
        if (fabs(hi - s->h) > 1e-12 * s->h) { free(s); return NULL; } /* cubic cells only */
    }
    double K1[MAXN * MAXN];
    or_basis(s->n, s->xi, s->w, s->D, s->F0, s->F1, K1, s->Atau, s->Kxi, s->L0, s->L1);
    s->Q = (double *)calloc((size_t)s->ncell * V * s->S, sizeof(double));
    return s;
}

void or_destroy(or_solver *s)
{
    if (!s) return;
    free(s->Q);
    free(s->cmat);
    free(s);
}

/* The state as held between traversals: each value rounded to the storage
 * precision. */
static void store_round(const or_solver *s, double *Q, size_t count)
{
    if (s->c.storage == OR_FP64) return;
    for (size_t i = 0; i < count; i++) Q[i] = or_round(s->c.storage, Q[i]);
}

void or_set_state(or_solver *s, const double *Q)
{
    const size_t count = (size_t)s->ncell * s->V * s->S;
    memcpy(s->Q, Q, count * sizeof(double));
    store_round(s, s->Q, count);
}

void or_get_state(const or_solver *s, double *Q)
{
    memcpy(Q, s->Q, (size_t)s->ncell * s->V * s->S * sizeof(double));
}

int or_set_material(or_solver *s, const double *c_per_cell)
{
    if (s->c.pde != OR_ACOUSTIC) return -1;
    if (!s->cmat) s->cmat = (double *)malloc((size_t)s->ncell * sizeof(double));
    memcpy(s->cmat, c_per_cell, (size_t)s->ncell * sizeof(double));
    return 0;
}

/* Point source s(t) delta(x - xs) in the first (pressure) equation.  Its
 * Galerkin projection onto the nodal basis of the cell holding xs is
 * s(t) phi_k(xs) / (h^d W_k) (W_k = product of Gauss weights).             */
int or_set_source(or_solver *s, const double *x, double f0, double t0, double amp)
{
    if (s->c.pde != OR_ACOUSTIC || s->c.predictor != OR_PICARD) return -1;
    int64_t cell = 0, m = 1;
    double loc[3];
    for (int i = 0; i < s->d; i++) {
        double u = (x[i] - s->c.lo[i]) / s->h;
        int ci = (int)floor(u);
        if (ci < 0 || ci >= s->c.cells[i]) return -1;
        loc[i] = u - ci;
        cell += ci * m;
        m *= s->c.cells[i];
    }
    double psi[3][MAXN];
    for (int i = 0; i < s->d; i++) lagrange_eval(s->n, s->xi, loc[i], psi[i]);
    double hd = pow(s->h, s->d);
    for (int sn = 0; sn < s->S; sn++) {
        double phi = 1.0, W = 1.0;
        for (int i = 0; i < s->d; i++) {
            int k = coord(sn, i, s->n);
            phi *= psi[i][k];
            W *= s->w[k];
        }
        s->src_phi[sn] = phi / (hd * W);
    }
    s->src_cell = cell;
    s->src_f0 = f0;
    s->src_t0 = t0;
    s->src_amp = amp;
    s->src_on = 1;
    return 0;
}

double or_max_eig(const or_solver *s)
{
    double lmax = 0.0;
    for (int64_t c = 0; c < s->ncell; c++)
        for (int sn = 0; sn < s->S; sn++) {
            double q[MAXV];
            for (int v = 0; v < s->V; v++) q[v] = s->Q[(c * s->V + v) * s->S + sn];
            for (int j = 0; j < s->d; j++) {
                double l = pde_max_eig(s, c, q, j);
                if (l > lmax) lmax = l;
            }
        }
    return lmax;
}

/* Time step of eq. CFL_condition for the given factor C_CFL. */
double or_max_dt(const or_solver *s, double cfl)
{
    return cfl * s->h / (s->d * (2.0 * s->c.order + 1.0) * or_max_eig(s));
}

/* ------------------------------------------------------------------------ */
/* Predictor (eq. Picard), per cell.                                          */
/*                                                                            */
/* Mapping the space-time cell to [0,1]^d x [0,1] and using Gauss quadrature  */
/* at the nodes (exact for these products), eq. Picard becomes, per spatial   */
/* node s:  K1 q_{.,s} = psi(0) Q_s - dt W R_{.,s}, where R_b = (1/h) sum_j   */
/* D_j F_j(q_b) [+ non-conservative part - source].  Since K1^{-1} psi(0) is  */
/* the vector of ones, the fixed-point form is                                */
/*     q_a <- Q - dt sum_b Atau[a][b] R_b(q),   a = 0..N,                      */
/* iterated I times from q_a = Q.                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *q, *qn, *Fj, *R, *eta, *deta, *tmp; /* scratch */
} cell_work;

static void work_alloc(const or_solver *s, cell_work *w)
{
    size_t VS = (size_t)s->V * s->S;
    w->q = (double *)malloc(sizeof(double) * s->n * VS);
    w->qn = (double *)malloc(sizeof(double) * s->n * VS);
    w->Fj = (double *)malloc(sizeof(double) * s->d * VS);
    w->R = (double *)malloc(sizeof(double) * s->n * VS);
    w->eta = (double *)malloc(sizeof(double) * s->S);
    w->deta = (double *)malloc(sizeof(double) * s->S);
    w->tmp = (double *)malloc(sizeof(double) * VS);
}

static void work_free(cell_work *w)
{
    free(w->q); free(w->qn); free(w->Fj); free(w->R);
    free(w->eta); free(w->deta); free(w->tmp);
}

/* R(q_b) at one time slice, in the predictor's precision. */
static void slice_residual(const or_solver *s, int64_t cell, const double *qb, double tb,
                           cell_work *w, double *R)
{
    const int S = s->S, V = s->V, d = s->d, p = s->c.prec[0];
    const double inv_h = 1.0 / s->h;
    /* pointwise fluxes; in emulated mode evaluated on FP32-rounded states and
     * rounded to p as contraction inputs */
    for (int sn = 0; sn < S; sn++) {
        double q[MAXV], F[MAXV];
        for (int v = 0; v < V; v++) q[v] = (p == OR_FP64) ? qb[v * S + sn] : or_round(OR_FP32, qb[v * S + sn]);
        for (int j = 0; j < d; j++) {
            pde_flux(s, cell, q, j, F);
            for (int v = 0; v < V; v++) w->Fj[(j * V + v) * S + sn] = F[v];
        }
    }
    /* divergence: sum over directions of D applied along that direction; in
     * emulated precision the sum over directions belongs to the same FP32
     * accumulation as the contraction itself */
    for (int i = 0; i < V * S; i++) R[i] = 0.0;
    for (int j = 0; j < d; j++) {
        apply_dir(s, s->D, j, w->Fj + (size_t)j * V * S, w->tmp, V, p);
        for (int i = 0; i < V * S; i++)
            R[i] = (p == OR_FP64) ? R[i] + w->tmp[i] : (double)((float)R[i] + (float)w->tmp[i]);
    }
    if (s->c.pde == OR_SWE) {
        for (int sn = 0; sn < S; sn++) {
            double hv = qb[0 * S + sn], bv = qb[3 * S + sn];
            if (p != OR_FP64) { hv = or_round(OR_FP32, hv); bv = or_round(OR_FP32, bv); }
            w->eta[sn] = hv + bv;
            if (p != OR_FP64) w->eta[sn] = or_round(OR_FP32, w->eta[sn]);
        }
        for (int j = 0; j < d; j++) {
            apply_dir(s, s->D, j, w->eta, w->deta, 1, p);
            for (int sn = 0; sn < S; sn++) {
                double hv = qb[0 * S + sn], nc[MAXV];
                if (p != OR_FP64) hv = or_round(OR_FP32, hv);
                swe_ncp(s, hv, w->deta[sn], j, nc);
                for (int v = 0; v < V; v++) {
                    double t = nc[v];
                    if (p != OR_FP64) t = or_round(OR_FP32, t);
                    R[v * S + sn] += t;
                }
            }
        }
    }
    for (int i = 0; i < V * S; i++) R[i] *= inv_h;
    if (s->src_on && cell == s->src_cell) {
        double st = ricker(s, tb);
        for (int sn = 0; sn < S; sn++) R[0 * S + sn] -= st * s->src_phi[sn];
    }
}

/* Space-time predictor of one cell.  Outputs (any may be NULL):
 *   qst  [n][V][S]  final Picard iterate at the n time nodes
 *   qbar [V][S]     time average sum_a w_a q_a                 (FP64)
 *   fbar [d][V][S]  time averages sum_a w_a F_j(q_a)           (FP64)
 *   nbar [V][S]     time average of sum_j B_j(q_a) D_j q_a     (FP64; SWE) */
/* Cauchy-Kowalevskaya predictor of one cell (linear flux, no source): with
 * dq/dt = -R(q) (R the spatial divergence of slice_residual), the Taylor terms
 * T_k = dt^k/k! d^kq/dt^k follow from T_0 = Q, T_k = -(dt/k) R(T_{k-1}),
 * k = 1..N.  The cell-local solution is q(t + tau dt) = sum_k T_k tau^k, its
 * time average over the step sum_k T_k / (k+1), and (linear flux) the flux
 * average F_j of that average.  Outputs as for predict(); qst holds the
 * expansion at the n time nodes. */
static void predict_ck(const or_solver *s, int64_t cell, const double *Q, double t, double dt,
                       cell_work *w, double *qst, double *qbar, double *fbar, double *nbar)
{
    const int n = s->n, S = s->S, V = s->V, d = s->d;
    const size_t VS = (size_t)V * S;
    double *T = w->q;                /* all n Taylor terms, [k][V][S] */
    memcpy(T, Q, VS * sizeof(double));
    for (int k = 1; k < n; k++) {
        slice_residual(s, cell, T + (k - 1) * VS, t, w, w->R);
        for (size_t i = 0; i < VS; i++) T[k * VS + i] = -(dt / k) * w->R[i];
    }
    double *avg = w->qn;
    for (size_t i = 0; i < VS; i++) {
        double acc = 0.0;
        for (int k = 0; k < n; k++) acc += T[k * VS + i] / (k + 1);
        avg[i] = acc;
    }
    if (qst)
        for (int a = 0; a < n; a++)
            for (size_t i = 0; i < VS; i++) {
                double acc = 0.0, tp = 1.0;
                for (int k = 0; k < n; k++) { acc += T[k * VS + i] * tp; tp *= s->xi[a]; }
                qst[a * VS + i] = acc;
            }
    if (qbar) memcpy(qbar, avg, VS * sizeof(double));
    if (fbar)
        for (int sn = 0; sn < S; sn++) {
            double q[MAXV], F[MAXV];
            for (int v = 0; v < V; v++) q[v] = avg[v * S + sn];
            for (int j = 0; j < d; j++) {
                pde_flux(s, cell, q, j, F);
                for (int v = 0; v < V; v++) fbar[(j * V + v) * S + sn] = F[v];
            }
        }
    if (nbar) memset(nbar, 0, sizeof(double) * VS);
}

static void predict(const or_solver *s, int64_t cell, const double *Q, double t, double dt,
                    cell_work *w, double *qst, double *qbar, double *fbar, double *nbar)
{
    const int n = s->n, S = s->S, V = s->V, d = s->d;
    const size_t VS = (size_t)V * S;
    if (s->c.predictor == OR_CK) {
        predict_ck(s, cell, Q, t, dt, w, qst, qbar, fbar, nbar);
        return;
    }
    for (int a = 0; a < n; a++) memcpy(w->q + a * VS, Q, VS * sizeof(double));
    for (int r = 0; r < s->I; r++) {
        for (int b = 0; b < n; b++)
            slice_residual(s, cell, w->q + b * VS, t + s->xi[b] * dt, w, w->R + b * VS);
        for (int a = 0; a < n; a++)
            for (size_t i = 0; i < VS; i++) {
                double acc = 0.0;
                for (int b = 0; b < n; b++) acc += s->Atau[a * n + b] * w->R[b * VS + i];
                w->qn[a * VS + i] = Q[i] - dt * acc;
            }
        double *t_ = w->q; w->q = w->qn; w->qn = t_;
    }
    if (qst) memcpy(qst, w->q, n * VS * sizeof(double));
    if (qbar) {
        for (size_t i = 0; i < VS; i++) {
            double acc = 0.0;
            for (int a = 0; a < n; a++) acc += s->w[a] * w->q[a * VS + i];
            qbar[i] = acc;
        }
    }
    if (fbar) {
        memset(fbar, 0, sizeof(double) * d * VS);
        for (int a = 0; a < n; a++)
            for (int sn = 0; sn < S; sn++) {
                double q[MAXV], F[MAXV];
                for (int v = 0; v < V; v++) q[v] = w->q[a * VS + v * S + sn];
                for (int j = 0; j < d; j++) {
                    pde_flux(s, cell, q, j, F);
                    for (int v = 0; v < V; v++) fbar[(j * V + v) * S + sn] += s->w[a] * F[v];
                }
            }
    }
    if (nbar) {
        memset(nbar, 0, sizeof(double) * VS);
        if (s->c.pde == OR_SWE) {
            for (int a = 0; a < n; a++) {
                const double *qa = w->q + a * VS;
                for (int sn = 0; sn < S; sn++) w->eta[sn] = qa[0 * S + sn] + qa[3 * S + sn];
                for (int j = 0; j < d; j++) {
                    apply_dir(s, s->D, j, w->eta, w->deta, 1, OR_FP64);
                    for (int sn = 0; sn < S; sn++) {
                        double nc[MAXV];
                        swe_ncp(s, qa[0 * S + sn], w->deta[sn], j, nc);
                        for (int v = 0; v < V; v++) nbar[v * S + sn] += s->w[a] * nc[v];
                    }
                }
            }
        }
    }
}

int or_predict_cell(const or_solver *s, int64_t cell, double t, double dt, double *qst,
                    double *qbar, double *fbar, double *nbar)
{
    if (cell < 0 || cell >= s->ncell) return -1;
    cell_work w;
    work_alloc(s, &w);
    predict(s, cell, s->Q + cell * s->V * s->S, t, dt, &w, qst, qbar, fbar, nbar);
    work_free(&w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Per-cell part of the corrector's first sweep: face projections (Alg. 1,    */
/* "expansion") and the volume integral.                                      */
/* Face arrays per cell: [d][side][V][F], side 0 at xi_j = 0, side 1 at 1.    */
/* ------------------------------------------------------------------------ */

static void cell_first_sweep(const or_solver *s, int64_t cell, double t, double dt, cell_work *w,
                             double *Qstar, double *fq, double *ff)
{
    const int n = s->n, S = s->S, V = s->V, d = s->d, F = s->F;
    const size_t VS = (size_t)V * S;
    const double *Q = s->Q + cell * VS;
    double *qbar = (double *)malloc(sizeof(double) * VS);
    double *fbar = (double *)malloc(sizeof(double) * d * VS);
    double *nbar = (double *)malloc(sizeof(double) * VS);
    predict(s, cell, Q, t, dt, w, NULL, qbar, fbar, nbar);

    if (fq) {
        const int p = s->c.prec[2];
        for (int j = 0; j < d; j++) {
            int st = stride_of(j, n);
            for (int side = 0; side < 2; side++) {
                const double *E = side ? s->F1 : s->F0;
                for (int v = 0; v < V; v++)
                    for (int sn = 0; sn < S; sn++) {
                        if (coord(sn, j, n) != 0) continue; /* one line per face node */
                        int f = face_of(sn, j, n, d);
                        size_t o = (((size_t)j * 2 + side) * V + v) * F + f;
                        fq[o] = or_round(p, contract(n, E, qbar + v * S + sn, st, p));
                        ff[o] = or_round(p, contract(n, E, fbar + ((size_t)j * V + v) * S + sn, st, p));
                    }
            }
        }
    }
    if (Qstar) {
        const double sigma = dt / s->h;
        const int p = s->c.prec[1];
        for (size_t i = 0; i < VS; i++) Qstar[i] = Q[i];
        for (int j = 0; j < d; j++) {
            apply_dir(s, s->Kxi, j, fbar + (size_t)j * VS, w->tmp, V, p);
            for (size_t i = 0; i < VS; i++) Qstar[i] += sigma * w->tmp[i];
        }
        if (s->c.pde == OR_SWE)
            for (size_t i = 0; i < VS; i++) Qstar[i] -= sigma * nbar[i];
        if (s->src_on && cell == s->src_cell) {
            double sbar = 0.0;
            for (int a = 0; a < n; a++) sbar += s->w[a] * ricker(s, t + s->xi[a] * dt);
            for (int sn = 0; sn < S; sn++) Qstar[0 * S + sn] += dt * sbar * s->src_phi[sn];
        }
    }
    free(qbar); free(fbar); free(nbar);
}

/* Numerical flux at one face node between left state (-) and right state (+)
 * in direction j.  G is the Rusanov flux (eq. rusanov_flux); for shallow water
 * the dissipation acts on the surface eta = h + b (eq. swe_custom_riemann) and
 * Dq is the path-conservative fluctuation 0.5 * B(midpoint) (q+ - q-), which
 * enters the left cell as G + Dq and the right cell as G - Dq.              */
static void riemann(const or_solver *s, int64_t cl, int64_t cr, int j, const double *qm,
                    const double *fm, const double *qp, const double *fp, double *G, double *Dq)
{
    const int V = s->V;
    double sl = pde_max_eig(s, cl, qm, j), sr = pde_max_eig(s, cr, qp, j);
    double sp = sl > sr ? sl : sr;
    for (int v = 0; v < V; v++) {
        G[v] = 0.5 * (fm[v] + fp[v]) - 0.5 * sp * (qp[v] - qm[v]);
        Dq[v] = 0.0;
    }
    if (s->c.pde == OR_SWE) {
        double deta = (qp[0] + qp[3]) - (qm[0] + qm[3]);
        G[0] = 0.5 * (fm[0] + fp[0]) - 0.5 * sp * deta;
        G[3] = 0.5 * (fm[3] + fp[3]);
        Dq[1 + j] = 0.5 * s->c.params[0] * 0.5 * (qm[0] + qp[0]) * deta;
    }
}

/* Face integral of one face into cell `cell` (eq. weak_form_volume_surface,
 * surface term): Q += sign * sigma * Lside[s_j] * Gface[f(s)].              */
static void lift(const or_solver *s, double *Q, int j, int side, const double *Gface, double sigma)
{
    const int n = s->n, S = s->S, V = s->V, F = s->F, d = s->d, p = s->c.prec[2];
    const double *L = side ? s->L1 : s->L0;
    const double sign = side ? -1.0 : 1.0;
    for (int v = 0; v < V; v++)
        for (int sn = 0; sn < S; sn++) {
            int f = face_of(sn, j, n, d);
            double lv = L[coord(sn, j, n)], g = Gface[v * F + f];
            double prod;
            if (p == OR_FP64) prod = lv * g;
            else prod = (double)((float)or_round(p, lv) * (float)or_round(p, g));
            Q[v * S + sn] += sign * sigma * prod;
        }
}

/* Corrector of one cell (second sweep of Alg. 1): Riemann solve on each of
 * its 2d faces and the face integral into the cell.  blk_q/blk_f hold 1+2d
 * pointers to face blocks [d][2][V][F]: entry 0 is the cell itself, entry
 * 1+2j+side the neighbour across direction j (side 0: lower, 1: upper).   */
static void correct_cell(const or_solver *s, int64_t cell, double dt, const double *const *blk_q,
                         const double *const *blk_f, double *Qc)
{
    const int V = s->V, d = s->d, F = s->F, p = s->c.prec[2];
    const double sigma = dt / s->h;
    double G[MAXV], Dq[MAXV], qm[MAXV], fm[MAXV], qp[MAXV], fpv[MAXV];
    double *Gface = (double *)malloc(sizeof(double) * V * F);
    for (int j = 0; j < d; j++)
        for (int side = 0; side < 2; side++) {
            int64_t nb = neighbour(s, cell, j, side ? +1 : -1);
            int64_t cl = side ? cell : nb, cr = side ? nb : cell;
            int kl = side ? 0 : 1 + 2 * j + side, kr = side ? 1 + 2 * j + side : 0;
            const double *Lq = blk_q[kl] + ((size_t)j * 2 + 1) * V * F;
            const double *Lf = blk_f[kl] + ((size_t)j * 2 + 1) * V * F;
            const double *Rq = blk_q[kr] + ((size_t)j * 2 + 0) * V * F;
            const double *Rf = blk_f[kr] + ((size_t)j * 2 + 0) * V * F;
            for (int f = 0; f < F; f++) {
                for (int v = 0; v < V; v++) {
                    qm[v] = Lq[v * F + f]; fm[v] = Lf[v * F + f];
                    qp[v] = Rq[v * F + f]; fpv[v] = Rf[v * F + f];
                }
                riemann(s, cl, cr, j, qm, fm, qp, fpv, G, Dq);
                for (int v = 0; v < V; v++) {
                    double g = side ? G[v] + Dq[v] : G[v] - Dq[v];
                    Gface[v * F + f] = (p == OR_FP64) ? g : or_round(OR_FP32, g);
                }
            }
            lift(s, Qc, j, side, Gface, sigma);
        }
    free(Gface);
}

/* One full time step t -> t + dt over every cell (Alg. 1). */
static int step_paper(or_solver *s, double t, double dt);

int or_step(or_solver *s, double t, double dt)
{
    if (s->c.semantics == OR_SEM_PAPER) return step_paper(s, t, dt);
    const size_t VS = (size_t)s->V * s->S;
    const size_t FS = (size_t)s->d * 2 * s->V * s->F;
    double *Qn = (double *)malloc(sizeof(double) * s->ncell * VS);
    double *fq = (double *)malloc(sizeof(double) * s->ncell * FS);
    double *ff = (double *)malloc(sizeof(double) * s->ncell * FS);
    if (!Qn || !fq || !ff) { free(Qn); free(fq); free(ff); return -1; }
#pragma omp parallel
    {
        cell_work w;
        work_alloc(s, &w);
#pragma omp for schedule(dynamic, 4)
        for (int64_t c = 0; c < s->ncell; c++) {
            cell_first_sweep(s, c, t, dt, &w, Qn + c * VS, fq + c * FS, ff + c * FS);
            store_round(s, Qn + c * VS, VS); /* Q* is stored between the traversals */
        }
        work_free(&w);
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < s->ncell; c++) {
        const double *bq[1 + 2 * 3], *bf[1 + 2 * 3];
        bq[0] = fq + c * FS;
        bf[0] = ff + c * FS;
        for (int j = 0; j < s->d; j++)
            for (int side = 0; side < 2; side++) {
                int64_t nc = neighbour(s, c, j, side ? +1 : -1);
                bq[1 + 2 * j + side] = fq + nc * FS;
                bf[1 + 2 * j + side] = ff + nc * FS;
            }
        correct_cell(s, c, dt, bq, bf, Qn + c * VS);
        store_round(s, Qn + c * VS, VS);
    }
    free(fq);
    free(ff);
    free(s->Q);
    s->Q = Qn;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Paper semantics (Sec. 4.1, Sec. 7): each kernel computes in its own type.  */
/* Every arithmetic result inside a kernel is rounded to the kernel's type p  */
/* (one rounding per operation, no fused multiply-add; constants and inputs   */
/* converted to p first).  Written out separately from the FP64 step above so */
/* that its rounding points can be read off line by line.                     */
/* ------------------------------------------------------------------------ */

static double rp(int p, double x) { return or_round(p, x); }
static double add_p(int p, double a, double b) { return rp(p, a + b); }
static double sub_p(int p, double a, double b) { return rp(p, a - b); }
static double mul_p(int p, double a, double b) { return rp(p, a * b); }
static double div_p(int p, double a, double b) { return rp(p, a / b); }

/* Physical flux F_j(q) with every operation in type p (q already in p). */
static void paper_flux(const or_solver *s, int64_t cell, const double *q, int j, int p, double *F)
{
    const int d = s->d;
    const double *pr = s->c.params;
    switch (s->c.pde) {
    case OR_ACOUSTIC: {
        double rho = rp(p, pr[0]), K = rp(p, cell_bulk(s, cell));
        F[0] = mul_p(p, K, q[1 + j]);
        for (int i = 0; i < d; i++) F[1 + i] = (i == j) ? div_p(p, q[0], rho) : 0.0;
        break;
    }
    case OR_ELASTIC: {
        double rho = rp(p, pr[0]), lam = rp(p, pr[1]), mu = rp(p, pr[2]);
        double l2m = add_p(p, lam, mul_p(p, rp(p, 2.0), mu));
        int ns = d * (d + 1) / 2;
        const double *v = q + ns;
        for (int a = 0; a < d; a++)
            for (int b = a; b < d; b++) {
                int k = stress_index(d, a, b);
                if (a == b)
                    F[k] = -mul_p(p, a == j ? l2m : lam, v[j]);
                else
                    F[k] = (b == j) ? -mul_p(p, mu, v[a]) : ((a == j) ? -mul_p(p, mu, v[b]) : 0.0);
            }
        for (int i = 0; i < d; i++) F[ns + i] = -div_p(p, q[stress_index(d, i, j)], rho);
        break;
    }
    case OR_EULER: {
        double g = rp(p, pr[0]), rho = q[0], E = q[1 + d];
        double ke = 0.0;
        for (int i = 0; i < d; i++) ke = add_p(p, ke, mul_p(p, q[1 + i], q[1 + i]));
        double pres = mul_p(p, sub_p(p, g, 1.0), sub_p(p, E, div_p(p, mul_p(p, 0.5, ke), rho)));
        double uj = div_p(p, q[1 + j], rho);
        F[0] = q[1 + j];
        for (int i = 0; i < d; i++) F[1 + i] = (i == j) ? add_p(p, mul_p(p, q[1 + i], uj), pres)
                                                          : mul_p(p, q[1 + i], uj);
        F[1 + d] = mul_p(p, uj, add_p(p, E, pres));
        break;
    }
    case OR_SWE: {
        double uj = div_p(p, q[1 + j], q[0]);
        F[0] = q[1 + j];
        F[1] = mul_p(p, q[1], uj);
        F[2] = mul_p(p, q[2], uj);
        F[3] = 0.0;
        break;
    }
    }
}

static double paper_max_eig(const or_solver *s, int64_t cell, const double *q, int j, int p)
{
    const int d = s->d;
    const double *pr = s->c.params;
    switch (s->c.pde) {
    case OR_ACOUSTIC: return rp(p, sqrt(div_p(p, rp(p, cell_bulk(s, cell)), rp(p, pr[0]))));
    case OR_ELASTIC:
        return rp(p, sqrt(div_p(p, add_p(p, rp(p, pr[1]), mul_p(p, 2.0, rp(p, pr[2]))), rp(p, pr[0]))));
    case OR_EULER: {
        double g = rp(p, pr[0]), rho = q[0], E = q[1 + d], ke = 0.0;
        for (int i = 0; i < d; i++) ke = add_p(p, ke, mul_p(p, q[1 + i], q[1 + i]));
        double pres = mul_p(p, sub_p(p, g, 1.0), sub_p(p, E, div_p(p, mul_p(p, 0.5, ke), rho)));
        return add_p(p, fabs(div_p(p, q[1 + j], rho)), rp(p, sqrt(div_p(p, mul_p(p, g, pres), rho))));
    }
    case OR_SWE: return add_p(p, fabs(div_p(p, q[1 + j], q[0])), rp(p, sqrt(mul_p(p, rp(p, pr[0]), q[0]))));
    }
    return 0.0;
}

/* sum_k m[k] x[k*stride] in type p: m converted to p, each product and each
 * partial sum rounded. */
static double contract_p(int n, const double *m, const double *x, int stride, int p)
{
    double a = 0.0;
    for (int k = 0; k < n; k++) a = add_p(p, a, mul_p(p, rp(p, m[k]), x[k * stride]));
    return a;
}

static void apply_dir_p(const or_solver *s, const double *M, int j, const double *X, double *out, int nv, int p)
{
    const int n = s->n, S = s->S, st = stride_of(j, n);
    for (int v = 0; v < nv; v++)
        for (int sn = 0; sn < S; sn++) {
            int i = coord(sn, j, n);
            out[v * S + sn] = contract_p(n, M + i * n, X + v * S + (sn - i * st), st, p);
        }
}

/* R(q_b) = (1/h) (sum_j D_j F_j(q_b) + non-conservative product), type p. */
static void paper_residual(const or_solver *s, int64_t cell, const double *qb, int p, cell_work *w, double *R)
{
    const int S = s->S, V = s->V, d = s->d;
    const double inv_h = rp(p, 1.0 / s->h);
    for (int sn = 0; sn < S; sn++) {
        double q[MAXV], F[MAXV];
        for (int v = 0; v < V; v++) q[v] = qb[v * S + sn];
        for (int j = 0; j < d; j++) {
            paper_flux(s, cell, q, j, p, F);
            for (int v = 0; v < V; v++) w->Fj[(j * V + v) * S + sn] = F[v];
        }
    }
    for (int i = 0; i < V * S; i++) R[i] = 0.0;
    for (int j = 0; j < d; j++) {
        apply_dir_p(s, s->D, j, w->Fj + (size_t)j * V * S, w->tmp, V, p);
        for (int i = 0; i < V * S; i++) R[i] = add_p(p, R[i], w->tmp[i]);
    }
    if (s->c.pde == OR_SWE) {
        const double g = rp(p, s->c.params[0]);
        for (int sn = 0; sn < S; sn++) w->eta[sn] = add_p(p, qb[0 * S + sn], qb[3 * S + sn]);
        for (int j = 0; j < d; j++) {
            apply_dir_p(s, s->D, j, w->eta, w->deta, 1, p);
            for (int sn = 0; sn < S; sn++)
                R[(1 + j) * S + sn] = add_p(p, R[(1 + j) * S + sn], mul_p(p, mul_p(p, g, qb[0 * S + sn]), w->deta[sn]));
        }
    }
    for (int i = 0; i < V * S; i++) R[i] = mul_p(p, R[i], inv_h);
}

/* The predictor kernel of one cell in type pp (Picard loop in pq): reads the
 * stored state Q, writes the face projections fq/ff [d][2][V][F] (type pp) and
 * Q* = Q + sigma sum_j Kxi_j Fbar_j (- sigma Nbar) in type pp. */
static void paper_predictor(const or_solver *s, int64_t cell, double dt, int pp, int pq, cell_work *w,
                            double *Qstar, double *fq, double *ff)
{
    const int n = s->n, S = s->S, V = s->V, d = s->d, F = s->F;
    const size_t VS = (size_t)V * S;
    const double *Q = s->Q + cell * VS;
    /* Picard iteration in pq */
    double *Qq = w->tmp;  /* not used by paper_residual's first phase; copied below */
    double *Q0 = (double *)malloc(sizeof(double) * VS);
    for (size_t i = 0; i < VS; i++) Q0[i] = rp(pq, Q[i]);
    (void)Qq;
    const double dtq = rp(pq, dt);
    for (int a = 0; a < n; a++) memcpy(w->q + a * VS, Q0, VS * sizeof(double));
    for (int r = 0; r < s->I; r++) {
        for (int b = 0; b < n; b++) paper_residual(s, cell, w->q + b * VS, pq, w, w->R + b * VS);
        for (int a = 0; a < n; a++)
            for (size_t i = 0; i < VS; i++) {
                double acc = 0.0;
                for (int b = 0; b < n; b++) acc = add_p(pq, acc, mul_p(pq, rp(pq, s->Atau[a * n + b]), w->R[b * VS + i]));
                w->qn[a * VS + i] = sub_p(pq, Q0[i], mul_p(pq, dtq, acc));
            }
        double *t_ = w->q; w->q = w->qn; w->qn = t_;
    }
    /* the rest of the predictor kernel in pp: the iterate converted to pp */
    for (size_t i = 0; i < (size_t)n * VS; i++) w->q[i] = rp(pp, w->q[i]);
    double *qbar = (double *)calloc(VS, sizeof(double));
    double *fbar = (double *)calloc((size_t)d * VS, sizeof(double));
    double *nbar = (double *)calloc(VS, sizeof(double));
    for (int a = 0; a < n; a++) {
        const double wa = rp(pp, s->w[a]);
        const double *qa = w->q + a * VS;
        for (size_t i = 0; i < VS; i++) qbar[i] = add_p(pp, qbar[i], mul_p(pp, wa, qa[i]));
        for (int sn = 0; sn < S; sn++) {
            double q[MAXV], Fl[MAXV];
            for (int v = 0; v < V; v++) q[v] = qa[v * S + sn];
            for (int j = 0; j < d; j++) {
                paper_flux(s, cell, q, j, pp, Fl);
                for (int v = 0; v < V; v++) {
                    double *f = fbar + ((size_t)j * V + v) * S + sn;
                    *f = add_p(pp, *f, mul_p(pp, wa, Fl[v]));
                }
            }
        }
        if (s->c.pde == OR_SWE) {
            const double g = rp(pp, s->c.params[0]);
            for (int sn = 0; sn < S; sn++) w->eta[sn] = add_p(pp, qa[0 * S + sn], qa[3 * S + sn]);
            for (int j = 0; j < d; j++) {
                apply_dir_p(s, s->D, j, w->eta, w->deta, 1, pp);
                for (int sn = 0; sn < S; sn++) {
                    double *nb = nbar + (size_t)(1 + j) * S + sn;
                    *nb = add_p(pp, *nb, mul_p(pp, wa, mul_p(pp, mul_p(pp, g, qa[0 * S + sn]), w->deta[sn])));
                }
            }
        }
    }
    /* face projections (stored in pp) */
    for (int j = 0; j < d; j++) {
        int st = stride_of(j, n);
        for (int side = 0; side < 2; side++) {
            const double *E = side ? s->F1 : s->F0;
            for (int v = 0; v < V; v++)
                for (int sn = 0; sn < S; sn++) {
                    if (coord(sn, j, n) != 0) continue;
                    int f = face_of(sn, j, n, d);
                    size_t o = (((size_t)j * 2 + side) * V + v) * F + f;
                    fq[o] = contract_p(n, E, qbar + v * S + sn, st, pp);
                    ff[o] = contract_p(n, E, fbar + ((size_t)j * V + v) * S + sn, st, pp);
                }
        }
    }
    /* volume integral added to the state (pp) */
    const double sigma = rp(pp, dt / s->h);
    for (size_t i = 0; i < VS; i++) Qstar[i] = rp(pp, Q[i]);
    for (int j = 0; j < d; j++) {
        apply_dir_p(s, s->Kxi, j, fbar + (size_t)j * VS, w->tmp, V, pp);
        for (size_t i = 0; i < VS; i++) Qstar[i] = add_p(pp, Qstar[i], mul_p(pp, sigma, w->tmp[i]));
    }
    if (s->c.pde == OR_SWE)
        for (size_t i = 0; i < VS; i++) Qstar[i] = sub_p(pp, Qstar[i], mul_p(pp, sigma, nbar[i]));
    free(Q0); free(qbar); free(fbar); free(nbar);
}

/* The corrector kernel of one cell in type pc: Rusanov (well-balanced for
 * shallow water) flux at each face node from the face data (converted to pc)
 * and the face integral added to the stored Q* (converted to pc). */
static void paper_corrector(const or_solver *s, int64_t cell, double dt, int pc, const double *const *blk_q,
                            const double *const *blk_f, double *Qc)
{
    const int n = s->n, S = s->S, V = s->V, d = s->d, F = s->F;
    const double sigma = rp(pc, dt / s->h), half = 0.5;
    for (size_t i = 0; i < (size_t)V * S; i++) Qc[i] = rp(pc, Qc[i]);
    double qm[MAXV], fm[MAXV], qp[MAXV], fpv[MAXV], G[MAXV];
    double *Gface = (double *)malloc(sizeof(double) * V * F);
    for (int j = 0; j < d; j++)
        for (int side = 0; side < 2; side++) {
            int64_t nb = neighbour(s, cell, j, side ? +1 : -1);
            int64_t cl = side ? cell : nb, cr = side ? nb : cell;
            int kl = side ? 0 : 1 + 2 * j + side, kr = side ? 1 + 2 * j + side : 0;
            const double *Lq = blk_q[kl] + ((size_t)j * 2 + 1) * V * F;
            const double *Lf = blk_f[kl] + ((size_t)j * 2 + 1) * V * F;
            const double *Rq = blk_q[kr] + ((size_t)j * 2 + 0) * V * F;
            const double *Rf = blk_f[kr] + ((size_t)j * 2 + 0) * V * F;
            for (int f = 0; f < F; f++) {
                for (int v = 0; v < V; v++) {
                    qm[v] = rp(pc, Lq[v * F + f]); fm[v] = rp(pc, Lf[v * F + f]);
                    qp[v] = rp(pc, Rq[v * F + f]); fpv[v] = rp(pc, Rf[v * F + f]);
                }
                double sl = paper_max_eig(s, cl, qm, j, pc), sr = paper_max_eig(s, cr, qp, j, pc);
                double sp = sl > sr ? sl : sr;
                for (int v = 0; v < V; v++)
                    G[v] = sub_p(pc, mul_p(pc, half, add_p(pc, fm[v], fpv[v])),
                                 mul_p(pc, mul_p(pc, half, sp), sub_p(pc, qp[v], qm[v])));
                if (s->c.pde == OR_SWE) {
                    double deta = sub_p(pc, add_p(pc, qp[0], qp[3]), add_p(pc, qm[0], qm[3]));
                    G[0] = sub_p(pc, mul_p(pc, half, add_p(pc, fm[0], fpv[0])), mul_p(pc, mul_p(pc, half, sp), deta));
                    G[3] = mul_p(pc, half, add_p(pc, fm[3], fpv[3]));
                    double hbar = mul_p(pc, half, add_p(pc, qm[0], qp[0]));
                    double dq = mul_p(pc, mul_p(pc, mul_p(pc, half, rp(pc, s->c.params[0])), hbar), deta);
                    G[1 + j] = side ? add_p(pc, G[1 + j], dq) : sub_p(pc, G[1 + j], dq);
                }
                for (int v = 0; v < V; v++) Gface[v * F + f] = G[v];
            }
            const double *L = side ? s->L1 : s->L0;
            for (int v = 0; v < V; v++)
                for (int sn = 0; sn < S; sn++) {
                    double t = mul_p(pc, sigma, mul_p(pc, rp(pc, L[coord(sn, j, n)]), Gface[v * F + face_of(sn, j, n, d)]));
                    Qc[v * S + sn] = side ? sub_p(pc, Qc[v * S + sn], t) : add_p(pc, Qc[v * S + sn], t);
                }
        }
    free(Gface);
}

static int step_paper(or_solver *s, double t, double dt)
{
    (void)t;
    const size_t VS = (size_t)s->V * s->S;
    const size_t FS = (size_t)s->d * 2 * s->V * s->F;
    const int pp = s->c.prec[0], pc = s->c.prec[2];
    const int pq = s->c.prec_picard >= 0 ? s->c.prec_picard : pp;
    double *Qn = (double *)malloc(sizeof(double) * s->ncell * VS);
    double *fq = (double *)malloc(sizeof(double) * s->ncell * FS);
    double *ff = (double *)malloc(sizeof(double) * s->ncell * FS);
    if (!Qn || !fq || !ff) { free(Qn); free(fq); free(ff); return -1; }
#pragma omp parallel
    {
        cell_work w;
        work_alloc(s, &w);
#pragma omp for schedule(dynamic, 4)
        for (int64_t c = 0; c < s->ncell; c++) {
            paper_predictor(s, c, dt, pp, pq, &w, Qn + c * VS, fq + c * FS, ff + c * FS);
            store_round(s, Qn + c * VS, VS);
        }
        work_free(&w);
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < s->ncell; c++) {
        const double *bq[1 + 2 * 3], *bf[1 + 2 * 3];
        bq[0] = fq + c * FS;
        bf[0] = ff + c * FS;
        for (int j = 0; j < s->d; j++)
            for (int side = 0; side < 2; side++) {
                int64_t nc = neighbour(s, c, j, side ? +1 : -1);
                bq[1 + 2 * j + side] = fq + nc * FS;
                bf[1 + 2 * j + side] = ff + nc * FS;
            }
        paper_corrector(s, c, dt, pc, bq, bf, Qn + c * VS);
        store_round(s, Qn + c * VS, VS);
    }
    free(fq);
    free(ff);
    free(s->Q);
    s->Q = Qn;
    return 0;
}

/* One step evaluated only at the listed cells (their new states written to
 * out[m][V][S]); the solver's own state is left unchanged.  Each listed cell
 * needs the first sweep of itself and of its 2d face neighbours.           */
int or_step_cells(const or_solver *s, double t, double dt, int m, const int64_t *ids, double *out)
{
    const size_t VS = (size_t)s->V * s->S;
    const size_t FS = (size_t)s->d * 2 * s->V * s->F;
    const int nb = 1 + 2 * s->d;
    int err = 0;
#pragma omp parallel
    {
        cell_work w;
        work_alloc(s, &w);
        double *fq = (double *)malloc(sizeof(double) * nb * FS);
        double *ff = (double *)malloc(sizeof(double) * nb * FS);
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < m; i++) {
            int64_t c = ids[i];
            if (c < 0 || c >= s->ncell) { err = -1; continue; }
            double *Qc = out + (size_t)i * VS;
            cell_first_sweep(s, c, t, dt, &w, Qc, fq, ff);
            store_round(s, Qc, VS);
            const double *bq[1 + 2 * 3], *bf[1 + 2 * 3];
            for (int k = 0; k < nb; k++) { bq[k] = fq + k * FS; bf[k] = ff + k * FS; }
            for (int j = 0; j < s->d; j++)
                for (int side = 0; side < 2; side++) {
                    int64_t nc = neighbour(s, c, j, side ? +1 : -1);
                    int k = 1 + 2 * j + side;
                    cell_first_sweep(s, nc, t, dt, &w, NULL, fq + k * FS, ff + k * FS);
                }
            correct_cell(s, c, dt, bq, bf, Qc);
            store_round(s, Qc, VS);
        }
        free(fq);
        free(ff);
        work_free(&w);
    }
    return err;
}

/* Receiver read-out: p_h(x_r) = sum_k phi_k(xi_r) Q_{0,k} in the cell holding x_r. */
int or_sample_points(const or_solver *s, int npts, const double *xyz, int var, double *out)
{
    for (int r = 0; r < npts; r++) {
        int64_t cell = 0, m = 1;
        double loc[3];
        for (int i = 0; i < s->d; i++) {
            double u = (xyz[r * 3 + i] - s->c.lo[i]) / s->h;
            int ci = (int)floor(u);
            if (ci < 0 || ci >= s->c.cells[i]) return -1;
            loc[i] = u - ci;
            cell += ci * m;
            m *= s->c.cells[i];
        }
        double psi[3][MAXN];
        for (int i = 0; i < s->d; i++) lagrange_eval(s->n, s->xi, loc[i], psi[i]);
        double acc = 0.0;
        for (int sn = 0; sn < s->S; sn++) {
            double phi = 1.0;
            for (int i = 0; i < s->d; i++) phi *= psi[i][coord(sn, i, s->n)];
            acc += phi * s->Q[(cell * s->V + var) * s->S + sn];
        }
        out[r] = acc;
    }
    return 0;
}

int or_info(const or_solver *s, int *out)
{
    out[0] = s->n; out[1] = s->d; out[2] = s->V; out[3] = s->S; out[4] = s->F; out[5] = s->I;
    out[6] = (int)s->ncell;
    return 0;
}

double or_cell_size(const or_solver *s) { return s->h; }

/* Number of OpenMP threads the parallel loops use. */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP loops from now on (timing the oracle on one core). */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint of one step for acoustics with per-cell sound speed.     */
/*                                                                            */
/* The step is affine in Q for fixed material (the point source adds a term  */
/* independent of Q, though not of the material).  This routine is          */
/* plain reverse mode over the forward operations of the step, in reverse    */
/* order, with every Picard iterate stored: face integral (lift), Rusanov    */
/* flux (including the speed s = max(c_L, c_R), ties to the left cell), face */
/* projection, volume integral, time averages, Picard iterations.  The bulk  */
/* modulus K = rho c^2 enters through F_j(q) = (K v_j, p/rho e_j).           */
/*   mu   <- (d Q^{n+1} / d Q^n)^T lam                                       */
/*   grad += d <lam, Q^{n+1}> / d c   (one entry per cell)                    */
/*                                                                            */
/* Mixed precision (predictor and volume formats both below FP64, flux FP64): */
/* the recomputed Picard iterates follow the forward step's emulation, and    */
/* each transposed contraction runs in the format of the forward contraction */
/* it transposes -- D_j^T of the Picard iterations in the predictor's format, */
/* Kxi^T of the volume integral in the volume format -- with the inputs       */
/* rounded to the format and FP32 accumulation (contract()).  The time        */
/* operator, the pointwise A_j^T, the face terms and every accumulation into  */
/* mu and grad stay FP64.  As the adjoint is linear in the incoming adjoint, */
/* each cell's contraction inputs are multiplied by a power of two before    */
/* the rounding and the results divided by it (exact operations), the power  */
/* chosen from the largest incoming adjoint value of the cell (lam and the   */
/* face terms G) so that it lands in [2^7, 2^8): the small adjoint values of */
/* a misfit sweep then keep the format's precision instead of underflowing   */
/* (FP16's smallest normal is 2^-14).  It approximates the exact adjoint to  */
/* the format's level; it is not the transpose of the rounded forward map,   */
/* which is not linear.                                                       */
/* ------------------------------------------------------------------------ */

/* y = A_j^T x at one node: A_j q = (K q[1+j], q[0]/rho e_j) */
#define ADJ_SCALE_EXP 8 /* scaled largest incoming adjoint value in [2^7, 2^8) */

/* apply_dir on sc * X (rounded in format p), result divided by sc; tmp: nv*S */
static void apply_dir_scaled(const or_solver *s, const double *M, int j, const double *X, double *out,
                             int nv, int p, double sc, double *tmp)
{
    const size_t m = (size_t)nv * s->S;
    for (size_t i = 0; i < m; i++) tmp[i] = sc * X[i];
    apply_dir(s, M, j, tmp, out, nv, p);
    for (size_t i = 0; i < m; i++) out[i] /= sc;
}

static void acoustic_flux_transpose(int d, double K, double rho, const double *x, int j, double *y)
{
    for (int v = 0; v <= d; v++) y[v] = 0.0;
    y[0] = x[1 + j] / rho;
    y[1 + j] = K * x[0];
}

int or_adjoint_step(or_solver *s, const double *Qn, double t, double dt, const double *lam,
                    double *mu, double *grad)
{
    if (s->c.pde != OR_ACOUSTIC || !s->cmat || s->c.predictor != OR_PICARD || s->c.storage != OR_FP64) return -1;
    const int pp = s->c.prec[0], pv = s->c.prec[1];
    if (s->c.prec[2] != OR_FP64 || (pp == OR_FP64) != (pv == OR_FP64)) return -1;
    const int n = s->n, S = s->S, V = s->V, d = s->d, F = s->F, I = s->I;
    const size_t VS = (size_t)V * S, FS = (size_t)d * 2 * V * F;
    const double rho = s->c.params[0], sigma = dt / s->h, inv_h = 1.0 / s->h;
    double Dt[MAXN * MAXN], Kxit[MAXN * MAXN], At[MAXN * MAXN];
    for (int i = 0; i < n; i++)
        for (int k = 0; k < n; k++) {
            Dt[i * n + k] = s->D[k * n + i];
            Kxit[i * n + k] = s->Kxi[k * n + i];
            At[i * n + k] = s->Atau[k * n + i];
        }
    /* forward: iterates (q^0..q^I) per cell, time average and face data */
    const size_t per_it = (size_t)n * VS;
    double *iters = (double *)malloc(sizeof(double) * s->ncell * (I + 1) * per_it);
    double *qbar = (double *)malloc(sizeof(double) * s->ncell * VS);
    double *fq = (double *)malloc(sizeof(double) * s->ncell * FS);
    if (!iters || !qbar || !fq) { free(iters); free(qbar); free(fq); return -1; }
    /* The point source adds a Q-independent term, but it reaches the later
     * Picard iterates and through them the K-dependent fluxes, so the
     * recomputed iterates keep it. */
#pragma omp parallel
    {
        cell_work w;
        work_alloc(s, &w);
#pragma omp for schedule(dynamic, 1)
        for (int64_t c = 0; c < s->ncell; c++) {
            const double *Qc = Qn + c * VS;
            double *it = iters + (size_t)c * (I + 1) * per_it;
            for (int a = 0; a < n; a++) memcpy(it + a * VS, Qc, VS * sizeof(double));
            for (int r = 0; r < I; r++) {
                double *qr = it + (size_t)r * per_it, *qn1 = it + (size_t)(r + 1) * per_it;
                for (int b = 0; b < n; b++)
                    slice_residual(s, c, qr + b * VS, t + s->xi[b] * dt, &w, w.R + b * VS);
                for (int a = 0; a < n; a++)
                    for (size_t i = 0; i < VS; i++) {
                        double acc = 0.0;
                        for (int b = 0; b < n; b++) acc += s->Atau[a * n + b] * w.R[b * VS + i];
                        qn1[a * VS + i] = Qc[i] - dt * acc;
                    }
            }
            const double *qI = it + (size_t)I * per_it;
            double *qb = qbar + c * VS;
            for (size_t i = 0; i < VS; i++) {
                double acc = 0.0;
                for (int a = 0; a < n; a++) acc += s->w[a] * qI[a * VS + i];
                qb[i] = acc;
            }
            for (int j = 0; j < d; j++) {
                int st = stride_of(j, n);
                for (int side = 0; side < 2; side++) {
                    const double *E = side ? s->F1 : s->F0;
                    for (int v = 0; v < V; v++)
                        for (int sn = 0; sn < S; sn++) {
                            if (coord(sn, j, n) != 0) continue;
                            int f = face_of(sn, j, n, d);
                            fq[c * FS + (((size_t)j * 2 + side) * V + v) * F + f] =
                                contract(n, E, qb + v * S + sn, st, OR_FP64);
                        }
                }
            }
        }
        work_free(&w);
    }
    /* reverse, per cell */
#pragma omp parallel
    {
        double *qbb = (double *)malloc(sizeof(double) * VS);      /* adjoint of qbar */
        double *fbb = (double *)malloc(sizeof(double) * d * VS);  /* adjoint of fbar_j */
        double *rho_a = (double *)malloc(sizeof(double) * n * VS);
        double *rho_n = (double *)malloc(sizeof(double) * n * VS);
        double *Rb = (double *)malloc(sizeof(double) * n * VS);
        double *Y = (double *)malloc(sizeof(double) * VS);
        double *T = (double *)malloc(sizeof(double) * VS);
        double *Gb = (double *)malloc(sizeof(double) * V * F);
#pragma omp for schedule(dynamic, 1)
        for (int64_t c = 0; c < s->ncell; c++) {
            const double *lc = lam + c * VS;
            const double K = rho * s->cmat[c] * s->cmat[c];
            double Kbar = 0.0;
            /* scale of the cell's contraction inputs (mixed precision) */
            double sc = 1.0;
            if (pp != OR_FP64) {
                double m = 0.0;
                for (size_t i = 0; i < VS; i++) m = fmax(m, fabs(lc[i]));
                for (int j = 0; j < d; j++) {
                    int st = stride_of(j, n);
                    for (int side = 0; side < 2; side++) {
                        int64_t nb = neighbour(s, c, j, side ? +1 : -1);
                        const double *lL = lam + (side ? c : nb) * VS, *lR = lam + (side ? nb : c) * VS;
                        for (int v = 0; v < V; v++)
                            for (int sn = 0; sn < S; sn++) {
                                if (coord(sn, j, n) != 0) continue;
                                double g = sigma * (contract(n, s->L0, lR + v * S + sn, st, OR_FP64) -
                                                    contract(n, s->L1, lL + v * S + sn, st, OR_FP64));
                                m = fmax(m, fabs(g));
                            }
                    }
                }
                if (m > 0.0) {
                    int e;
                    frexp(m, &e);
                    sc = ldexp(1.0, ADJ_SCALE_EXP - e);
                }
            }
            /* volume: Qstar += sigma sum_j Kxi (x)_j fbar_j */
            for (int j = 0; j < d; j++) {
                apply_dir_scaled(s, Kxit, j, lc, fbb + (size_t)j * VS, V, pv, sc, T);
                for (size_t i = 0; i < VS; i++) fbb[(size_t)j * VS + i] *= sigma;
            }
            memset(qbb, 0, sizeof(double) * VS);
            /* faces of this cell */
            for (int j = 0; j < d; j++) {
                int st = stride_of(j, n);
                for (int side = 0; side < 2; side++) {
                    int64_t nb = neighbour(s, c, j, side ? +1 : -1);
                    int64_t cl = side ? c : nb, cr = side ? nb : c;
                    const double *lL = lam + cl * VS, *lR = lam + cr * VS;
                    const double sl = s->cmat[cl], sr = s->cmat[cr];
                    const double sp = sl >= sr ? sl : sr;
                    const int c_is_max = side ? (sl >= sr) : (sr > sl);
                    double sbar = 0.0;
                    for (int v = 0; v < V; v++)
                        for (int sn = 0; sn < S; sn++) {
                            if (coord(sn, j, n) != 0) continue;
                            int f = face_of(sn, j, n, d);
                            /* adjoint of the face flux G: Q_L -= sigma L1 G, Q_R += sigma L0 G */
                            double g = sigma * (contract(n, s->L0, lR + v * S + sn, st, OR_FP64) -
                                                contract(n, s->L1, lL + v * S + sn, st, OR_FP64));
                            Gb[v * F + f] = g;
                            const double qm = fq[cl * FS + (((size_t)j * 2 + 1) * V + v) * F + f];
                            const double qp = fq[cr * FS + (((size_t)j * 2 + 0) * V + v) * F + f];
                            sbar += -0.5 * g * (qp - qm);
                        }
                    if (c_is_max) Kbar += sbar / (2.0 * rho * s->cmat[c]); /* ds/dK of s = sqrt(K/rho) */
                    /* G = 0.5 (f- + f+) - 0.5 s (q+ - q-): this cell's side */
                    const double *E = side ? s->F1 : s->F0;
                    const double qsign = side ? 0.5 * sp : -0.5 * sp;
                    for (int v = 0; v < V; v++)
                        for (int sn = 0; sn < S; sn++) {
                            int i = coord(sn, j, n), f = face_of(sn, j, n, d);
                            qbb[v * S + sn] += E[i] * qsign * Gb[v * F + f];
                            fbb[((size_t)j * V + v) * S + sn] += E[i] * 0.5 * Gb[v * F + f];
                        }
                }
            }
            /* fbar_j = A_j qbar */
            const double *qb = qbar + c * VS;
            for (int j = 0; j < d; j++)
                for (int sn = 0; sn < S; sn++) {
                    double x[MAXV], y[MAXV];
                    for (int v = 0; v < V; v++) x[v] = fbb[((size_t)j * V + v) * S + sn];
                    acoustic_flux_transpose(d, K, rho, x, j, y);
                    for (int v = 0; v < V; v++) qbb[v * S + sn] += y[v];
                    Kbar += x[0] * qb[(1 + j) * S + sn];
                }
            /* qbar = sum_a w_a q^I_a */
            double *mc = mu + c * VS;
            for (size_t i = 0; i < VS; i++) mc[i] = lc[i];
            for (int a = 0; a < n; a++)
                for (size_t i = 0; i < VS; i++) rho_a[a * VS + i] = s->w[a] * qbb[i];
            for (int a = 0; a < n; a++)
                for (size_t i = 0; i < VS; i++) mc[i] += rho_a[a * VS + i];
            /* Picard iterations in reverse: q^{r+1}_a = Q - dt sum_b Atau[a][b] R_b(q^r_b) */
            const double *it = iters + (size_t)c * (I + 1) * per_it;
            for (int r = I - 1; r >= 0; r--) {
                for (int b = 0; b < n; b++)
                    for (size_t i = 0; i < VS; i++) {
                        double acc = 0.0;
                        for (int a = 0; a < n; a++) acc += At[b * n + a] * rho_a[a * VS + i];
                        Rb[b * VS + i] = -dt * acc;
                    }
                memset(rho_n, 0, sizeof(double) * n * VS);
                const double *qr = it + (size_t)r * per_it;
                for (int b = 0; b < n; b++)
                    for (int j = 0; j < d; j++) {
                        /* R_b = (1/h) sum_j D_j A_j q_b */
                        apply_dir_scaled(s, Dt, j, Rb + b * VS, Y, V, pp, sc, T);
                        for (int sn = 0; sn < S; sn++) {
                            double x[MAXV], y[MAXV];
                            for (int v = 0; v < V; v++) x[v] = inv_h * Y[v * S + sn];
                            acoustic_flux_transpose(d, K, rho, x, j, y);
                            for (int v = 0; v < V; v++) rho_n[b * VS + v * S + sn] += y[v];
                            Kbar += x[0] * qr[b * VS + (1 + j) * S + sn];
                        }
                    }
                memcpy(rho_a, rho_n, sizeof(double) * n * VS);
                for (int a = 0; a < n; a++)
                    for (size_t i = 0; i < VS; i++) mc[i] += rho_a[a * VS + i];
            }
            grad[c] += Kbar * 2.0 * rho * s->cmat[c];
        }
        free(qbb); free(fbb); free(rho_a); free(rho_n); free(Rb); free(Y); free(T); free(Gb);
    }
    free(iters);
    free(qbar);
    free(fq);
    return 0;
}

/* Nodal weights of point x: out[node] = phi_node(x) in the cell holding x. */
int or_point_weights(const or_solver *s, const double *x, int64_t *cell_out, double *out)
{
    int64_t cell = 0, m = 1;
    double loc[3];
    for (int i = 0; i < s->d; i++) {
        double u = (x[i] - s->c.lo[i]) / s->h;
        int ci = (int)floor(u);
        if (ci < 0 || ci >= s->c.cells[i]) return -1;
        loc[i] = u - ci;
        cell += ci * m;
        m *= s->c.cells[i];
    }
    double psi[3][MAXN];
    for (int i = 0; i < s->d; i++) lagrange_eval(s->n, s->xi, loc[i], psi[i]);
    for (int sn = 0; sn < s->S; sn++) {
        double phi = 1.0;
        for (int i = 0; i < s->d; i++) phi *= psi[i][coord(sn, i, s->n)];
        out[sn] = phi;
    }
    *cell_out = cell;
    return 0;
}
