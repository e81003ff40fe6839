/*
 * FP64 CPU oracle of the ADER-DG time step (arXiv 2504.06889, Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg.  Independent of the GPU library (no shared
 * code, headers or tables).
 *
 * Layouts (all FP64, row-major):
 *   state      Q[cell][var][node], node = i0 + n*(i1 + n*i2) (x fastest),
 *              cell = c0 + C0*(c1 + C1*c2) (x fastest), n = order + 1.
 *   face block [dir][side][var][face node], side 0 at xi_dir = 0.
 *
 * Readings of points the paper leaves open:
 *   - Picard iteration count I = order+1 (config picard_iters = 0), fixed, from
 *     the initial guess q_a = Q^n at every time node a;
 *   - time basis: Gauss-Legendre nodes, as in space;
 *   - the Riemann solver acts once per face on the time averages of the face
 *     states and fluxes;
 *   - Rusanov speed: the larger |eigenvalue| of the two sides, per face node;
 *   - Euler energy flux v_j (E + p) with E the total energy per volume;
 *   - shallow water: conservative flux (h u_j, h u u_j, h v u_j, 0), the
 *     pressure term g h d(h+b) as the non-conservative product evaluated as
 *     g h D(eta) with eta = h + b; the Rusanov dissipation acts on (eta, hu,
 *     hv, 0) and the face fluctuation 0.5 g hbar (eta+ - eta-) enters the
 *     normal momentum (left cell: G + Dq, right cell: G - Dq);
 *   - point source (acoustics only): s(t) delta(x - xs) in the pressure
 *     equation, s a Ricker wavelet, included in predictor and corrector;
 *   - Cauchy-Kowalevskaya predictor (linear PDEs, the paper's alternative to
 *     the Picard iteration, Sec. 3): the Taylor expansion of the cell-local
 *     solution in time to degree N, its time derivatives taken from the PDE
 *     (d/dt = minus the discrete divergence, applied repeatedly); the time
 *     average of the truncated expansion replaces the Picard time average.
 *
 * Emulated precision (prec[0] predictor, prec[1] volume, prec[2] flux; values
 * OR_FP64/OR_FP32/OR_BF16/OR_FP16): the inputs of the contraction (data and
 * matrix) are rounded (FP32 first, then to the format, round-to-nearest-even),
 * products and sums in FP32 (for the predictor, the sum over the d directions
 * of the divergence too), result widened to FP64.  Pointwise fluxes of the
 * predictor then use FP32-rounded states; face values are stored rounded to
 * the flux format; the lift multiplies format-rounded inputs in FP32.  Time
 * averages, the Picard time operator and all state accumulation stay FP64.
 *
 * Paper semantics (semantics = OR_SEM_PAPER; Sec. 4.1, each generated kernel
 * computes in the type it is instantiated for): the predictor kernel (Picard
 * loop, time averages, face projection, volume integral and its addition to
 * the state) runs in prec[0], its Picard loop in prec_picard if that is set,
 * the corrector kernel (Riemann solve, face integral and its addition) in
 * prec[2]; every arithmetic result, constant and intermediate value inside a
 * kernel is rounded to the kernel's type (one rounding per operation, no fused
 * multiply-add), kernel inputs are converted to it and outputs are stored in
 * it, and the state between the kernels is held in the storage type.  prec[1]
 * is unused.  Picard predictor, 1-D to 3-D, no point source.
 *
 * Storage precision (the paper's fourth control, Sec. 4.1): the persistent
 * state is held in that format between grid traversals: the state given to
 * or_set_state, the first sweep's Q* and the corrected state are each rounded
 * to it (FP32 first, then the format); all arithmetic stays as above.
 */
#ifndef ADERDG_ORACLE_H
#define ADERDG_ORACLE_H

#include <stdint.h>

#define OR_MAXN 10
#define OR_MAXV 9

enum { OR_ACOUSTIC = 0, OR_ELASTIC = 1, OR_EULER = 2, OR_SWE = 3 };
enum { OR_FP64 = 0, OR_FP32 = 1, OR_BF16 = 2, OR_FP16 = 3 };
enum { OR_PICARD = 0, OR_CK = 1 };
enum { OR_SEM_BUILD = 0, OR_SEM_PAPER = 1 };

typedef struct {
    int dim, order;
    int cells[3];
    double lo[3], hi[3];
    int pde;
    double params[8]; /* acoustic: rho, K | elastic: rho, lambda, mu | euler: gamma | swe: g */
    int picard_iters; /* 0 -> order + 1 */
    int prec[3];      /* emulated precision: predictor, volume, flux */
    int predictor;    /* OR_PICARD, or OR_CK (linear PDEs without a point source) */
    int storage;      /* emulated storage precision of the state between traversals */
    int semantics;    /* OR_SEM_BUILD (contraction inputs rounded, FP32 accumulation) or
                         OR_SEM_PAPER (each kernel computes and stores in its type)   */
    int prec_picard;  /* paper semantics: type of the Picard loop (-1: the predictor's) */
} or_config;

typedef struct or_solver {
    or_config c;
    int n, d, V, S, F, I;
    int64_t ncell;
    double h;
    double xi[OR_MAXN], w[OR_MAXN], D[OR_MAXN * OR_MAXN], F0[OR_MAXN], F1[OR_MAXN];
    double Atau[OR_MAXN * OR_MAXN], Kxi[OR_MAXN * OR_MAXN], L0[OR_MAXN], L1[OR_MAXN];
    double *Q;
    double *cmat;
    int src_on;
    int64_t src_cell;
    double src_phi[OR_MAXN * OR_MAXN * OR_MAXN];
    double src_f0, src_t0, src_amp;
} or_solver;

double or_round(int p, double x);
int or_basis(int n, double *xi, double *w, double *D, double *F0, double *F1, double *K1,
             double *Atau, double *Kxi, double *L0, double *L1);
int or_nvars(int pde, int dim);

or_solver *or_create(const or_config *cfg);
void or_destroy(or_solver *s);
void or_set_state(or_solver *s, const double *Q);
void or_get_state(const or_solver *s, double *Q);
int or_set_material(or_solver *s, const double *c_per_cell);
int or_set_source(or_solver *s, const double *x, double f0, double t0, double amp);
double or_max_eig(const or_solver *s);
double or_max_dt(const or_solver *s, double cfl);
int or_predict_cell(const or_solver *s, int64_t cell, double t, double dt, double *qst,
                    double *qbar, double *fbar, double *nbar);
int or_step(or_solver *s, double t, double dt);
int or_step_cells(const or_solver *s, double t, double dt, int m, const int64_t *ids, double *out);
int or_sample_points(const or_solver *s, int npts, const double *xyz, int var, double *out);
int or_info(const or_solver *s, int *out);
double or_cell_size(const or_solver *s);
int or_num_threads(void);
void or_set_num_threads(int n);
int or_adjoint_step(or_solver *s, const double *Qn, double t, double dt, const double *lam,
                    double *mu, double *grad);
int or_point_weights(const or_solver *s, const double *x, int64_t *cell_out, double *out);

#endif
