/*
 * aderdg.h - C ABI of the MI355X (gfx950) ADER-DG time-step library.
 *
 * The library advances hyperbolic systems q_t + div F(q) + B(q) grad q = S on a
 * periodic Cartesian grid with the ADER-DG one-step scheme of arXiv 2504.06889,
 * Sec. 3: a cell-local space-time predictor (eq. Picard, solved by Picard
 * iteration), the volume integral and the surface integral of the Rusanov
 * numerical flux (eq. weak_form_volume_surface, eq. rusanov_flux), in the
 * order of Alg. 1.  Per-kernel precision follows Sec. 4.1 (the "predictor",
 * "corrector" and "storage" controls), remapped as described below.
 *
 * Conventions
 *  - Every call returns an aderdg_status; no C++ exception crosses the ABI.
 *    On failure aderdg_last_error() describes the cause.
 *  - The library owns all device memory it allocates (state, face buffers,
 *    material, scratch).  Caller pointers are borrowed: host data is copied
 *    before the call returns; device data is read or written in stream order
 *    on the solver's stream.  The library never frees caller memory.
 *  - All GPU work is enqueued on the hipStream_t given to aderdg_create (NULL:
 *    the default stream).  Calls on one solver must not overlap in time from
 *    several host threads.
 *  - State layout (host and device): Q[cell][var][node], FP64, with
 *    node = i0 + n*(i1 + n*i2) (x fastest), n = order + 1 Gauss-Legendre
 *    points per dimension, and cell = c0 + C0*(c1 + C1*c2) (x fastest).
 *  - Variables: acoustic (p, v_1..v_d); elastic 2-D (sxx, syy, sxy, vx, vy),
 *    3-D (sxx, syy, szz, sxy, syz, sxz, vx, vy, vz); Euler (rho, rho v_1..v_d,
 *    E); shallow water 2-D (h, hu, hv, b).
 */
#ifndef ADERDG_H
#define ADERDG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aderdg_solver aderdg_solver;

typedef enum {
    ADERDG_OK = 0,
    ADERDG_E_INVALID = -1,     /* bad argument or configuration                       */
    ADERDG_E_UNSUPPORTED = -2, /* valid but not built (order/PDE/dim/precision combo) */
    ADERDG_E_OOM = -3,         /* device allocation failed                            */
    ADERDG_E_DEVICE = -4,      /* a HIP runtime call failed                           */
    ADERDG_E_NONFINITE = -5    /* the state holds NaN or Inf                          */
} aderdg_status;

typedef enum { ADERDG_ACOUSTIC = 0, ADERDG_ELASTIC = 1, ADERDG_EULER = 2, ADERDG_SWE = 3 } aderdg_pde;

/* Kernels whose contractions take a precision (Sec. 4.1, four controls):
 *   PREDICTOR - the Picard iteration's spatial-derivative contractions (the
 *               paper's "predictor" and "Picard" controls; Picard is used for
 *               every PDE here);
 *   VOLUME    - the volume-integral contraction;
 *   FLUX      - face projection, face-value storage, Riemann solve and lift
 *               (the paper's "corrector"; the update Q += dt (...) stays FP64);
 *   STORAGE   - the format of the persistent state held in device memory
 *               between traversals (the state given to set_state, Q* after
 *               the predictor, the corrected state): FP64 (default), or
 *               FP32/BF16/FP16 elements (8/4/2 bytes, same layout), each
 *               value rounded to the format (FP32 first, then the format)
 *               when it is stored and widened exactly when it is read; all
 *               arithmetic is unchanged.  get/set_state still take FP64.
 * In a lower precision the contraction inputs (data and matrix) are rounded
 * to that format (round-to-nearest-even) and the products are accumulated in
 * FP32 (matrix cores for PREDICTOR and VOLUME in BF16/FP16, the vector ALU in
 * FP32); the Picard time operator, the
 * time-average weights and every accumulation into the state stay FP64.  */
typedef enum { ADERDG_K_PREDICTOR = 0, ADERDG_K_VOLUME = 1, ADERDG_K_FLUX = 2, ADERDG_K_STORAGE = 3 } aderdg_kernel;
typedef enum { ADERDG_FP64 = 0, ADERDG_FP32 = 1, ADERDG_BF16 = 2, ADERDG_FP16 = 3 } aderdg_prec;

/* Space-time predictor (Sec. 3): the Picard iteration of eq. Picard, or, for
 * linear PDEs, the Cauchy-Kowalevskaya procedure the paper names as the
 * cheaper alternative (time derivatives from the PDE, Taylor expansion to
 * degree N in time).                                                         */
typedef enum { ADERDG_PICARD = 0, ADERDG_CK = 1 } aderdg_predictor;

typedef struct {
    int dim;          /* 2 or 3 (shallow water: 2)                                    */
    int order;        /* polynomial order N (n = N+1 nodes per dimension)             */
    int cells[3];     /* cells per dimension (entries beyond dim ignored); the total
                         is at most 2^31 - 1                                          */
    double lo[3];     /* domain lower corner                                          */
    double hi[3];     /* domain upper corner; cells must be cubes (equal h)           */
    int pde;          /* aderdg_pde                                                   */
    double params[8]; /* acoustic: rho, K | elastic: rho, lambda, mu | Euler: gamma | SWE: g */
    int picard_iters; /* Picard iterations per step; 0 -> N+1                         */
} aderdg_config;

/* Create a solver (Sec. 3 scheme on the given grid).  Builds the
 * Gauss-Legendre basis and operators on the host in FP64, allocates the state
 * (zero), face buffers and constants on the current HIP device.  `hip_stream`
 * is a hipStream_t (may be NULL).  Errors: INVALID (bad config, 2^31 or more
 * cells, or NULL out),
 * UNSUPPORTED (order/PDE/dim not built), OOM, DEVICE.                        */
aderdg_status aderdg_create(const aderdg_config *cfg, void *hip_stream, aderdg_solver **out);

/* Synchronise the stream and release every device buffer.  NULL is a no-op. */
aderdg_status aderdg_destroy(aderdg_solver *s);

/* Copy a full state (layout above, cells*V*n^d doubles) into the solver.
 * is_device: 0 host pointer (synchronous copy), 1 device pointer (stream
 * ordered copy).  Clears the non-finite flag.                                */
aderdg_status aderdg_set_state(aderdg_solver *s, const double *Q, int is_device);

/* Copy the state out (same layout).  Synchronises the stream for host copies.
 * Returns NONFINITE (after copying) if any state value is NaN or Inf.        */
aderdg_status aderdg_get_state(aderdg_solver *s, double *Q, int is_device);

/* Per-cell sound speed c (acoustics only; K = rho c^2 per cell, Rusanov speed
 * max(c_L, c_R) at each face).  `c` holds one double per cell.               */
aderdg_status aderdg_set_material(aderdg_solver *s, const double *c, int is_device);

/* Select the space-time predictor (aderdg_predictor; default PICARD).  CK: the
 * Taylor terms T_0 = Q, T_k = -(dt/k) R(T_{k-1}) (R the divergence of the
 * cell-local fluxes, its contraction in the PREDICTOR precision) for
 * k = 1..N, time average sum_k T_k/(k+1) in FP64; face data and volume term
 * from that average as for Picard.  Errors: INVALID (unknown kind),
 * UNSUPPORTED (CK for a nonlinear PDE, or with a point source set).  The
 * adjoint and point sources need PICARD.                                      */
aderdg_status aderdg_set_predictor(aderdg_solver *s, int kind);

/* Select the precision of one kernel's contractions, or the storage precision
 * of the state (see aderdg_kernel).  Setting STORAGE moves the state held now
 * into a new buffer of that format, rounding each value (synchronises the
 * stream; the old buffer is freed).  Errors: INVALID (unknown
 * kernel/precision), UNSUPPORTED (predictor format not built), OOM, DEVICE.
 * The adjoint needs FP64 storage.                                            */
aderdg_status aderdg_set_precision(aderdg_solver *s, int kernel, int prec);

/* Largest admissible time step of eq. CFL_condition,
 * dt = cfl * h / (d (2N+1) lambda_max), lambda_max over all nodes and
 * directions of the current state.  Synchronises the stream.                */
aderdg_status aderdg_max_dt(aderdg_solver *s, double cfl, double *dt_out);

/* Advance the state by `nsteps` steps of size dt (Alg. 1: predictor with face
 * projection and volume integral per cell, then Riemann solve and face
 * integral per cell).  Asynchronous on the solver's stream; the solver's time
 * advances by nsteps*dt.  Errors: INVALID (dt <= 0, nsteps < 0).            */
aderdg_status aderdg_step(aderdg_solver *s, double dt, int nsteps);

/* Solver time (used by the point source).                                   */
aderdg_status aderdg_set_time(aderdg_solver *s, double t);
aderdg_status aderdg_get_time(const aderdg_solver *s, double *t);

/* Point source amp * ricker(t) * delta(x - xs) in the first (pressure) equation
 * (acoustics only; eq. exa_canonical_form's point-source term), ricker(t) =
 * (1 - 2 a) exp(-a), a = pi^2 f0^2 (t - t0)^2.  Projected onto the basis of the
 * cell holding xs; enters both the predictor and the volume update.        */
aderdg_status aderdg_set_source(aderdg_solver *s, const double x[3], double f0, double t0, double amp);

/* Receivers: nrec points xyz[nrec][3] where the first variable is sampled by
 * its nodal polynomial.  Replaces any previous set.                          */
aderdg_status aderdg_set_receivers(aderdg_solver *s, int nrec, const double *xyz);

/* Values of the first variable at the receivers for the current state;
 * out[nrec] (host or device).                                               */
aderdg_status aderdg_read_receivers(aderdg_solver *s, double *out, int is_device);

/* Adjoint of one step (acoustics with a per-cell material).  Given the
 * state Qn (device, the state at the start of the step), the adjoint lam
 * (device, state layout) of the state after the step, it overwrites lam with
 * the adjoint of Qn (the transpose of the step applied to lam) and adds to
 * grad (device, one double per cell) the derivative of <lam_in, step(Qn)>
 * with respect to each cell's sound speed.  The solver's own state is not
 * used or changed; dt must equal the forward step.
 * Precision: with PREDICTOR and VOLUME in FP64 everything is FP64; with both
 * in lower formats (dim 2 order 3, dim 3 orders 2 and 5) each transposed
 * contraction runs in the format of the forward one -- the derivative passes
 * of the Picard iterations in the predictor's format, the volume operator in
 * the volume format -- on rounded inputs with FP32 accumulation, everything
 * else in FP64: the exact adjoint to the format's level.
 * Errors: INVALID (null pointer, dt <= 0), UNSUPPORTED (not acoustics with a
 * material, CK predictor, storage or FLUX other than FP64, one of PREDICTOR
 * and VOLUME in FP64 and the other not, (dim, order) not built), OOM, DEVICE. */
aderdg_status aderdg_step_adjoint(aderdg_solver *s, double dt, double t, const double *Qn_dev,
                                  double *lam_dev, double *grad_dev);

/* The face data of the last step's predictor (the time-averaged q and F_j
 * projected to both sides of every face, Alg. 1 "expansion"), copied to dst
 * (device if is_device, else host; a host copy synchronises), info[7] bytes per
 * cell in the FLUX format: layout [cell][dir][side][q|f][var][face node], or,
 * for a linear PDE with FP64 faces, whose f halves the predictor does not write
 * (the corrector evaluates the flux from the projected q),
 * [cell][dir][side][var][face node] with the q halves only.  Valid after
 * aderdg_step; dst is owned by the caller.                                  */
aderdg_status aderdg_copy_faces(aderdg_solver *s, void *dst, int is_device);

/* aderdg_step_adjoint with the forward face data of the step supplied by the
 * caller (fwd_faces_dev: what aderdg_copy_faces returned right after the
 * forward step from Qn, FLUX FP64) instead of recomputed from Qn: the result
 * is identical, one predictor launch cheaper.  Errors as aderdg_step_adjoint. */
aderdg_status aderdg_step_adjoint_faces(aderdg_solver *s, double dt, double t, const double *Qn_dev,
                                        const void *fwd_faces_dev, double *lam_dev, double *grad_dev);

/* aderdg_step_adjoint_faces for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments and results, bit for bit, but the face
 * restrictions of the incoming adjoint go to a static device array of the
 * library (ADERDG_NOALLOC_SCRATCH_BYTES = 64 MiB on each GPU the library runs
 * on, held until the process ends) and no device memory is allocated or freed.
 * Limit: ncell * dim * 2 * (dim + 1) * (order + 1)^(dim - 1) * 8 bytes must not
 * exceed the array (e.g. 9709 cells of 3-D order 5).  Every call on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU (several
 * streams or threads) race and must be serialised by the caller.
 * Errors: INVALID (null pointer, dt <= 0, grid beyond the limit), the other
 * errors of aderdg_step_adjoint.                                              */
#define ADERDG_NOALLOC_SCRATCH_BYTES (64u << 20)
aderdg_status aderdg_step_adjoint_faces_noalloc(aderdg_solver *s, double dt, double t, const double *Qn_dev,
                                                const void *fwd_faces_dev, double *lam_dev, double *grad_dev);

/* Scatter the receiver misfit gradient (the transpose of the receiver
 * read-out): lam[cell][0][node] += sum_r weight[r] * phi_node(x_r) over the
 * receivers in that cell (device pointers: weight[nrec], lam in the state
 * layout).  Each cell's receivers are summed in a fixed order (by receiver
 * index), so repeated calls give bitwise-equal results.                     */
aderdg_status aderdg_receivers_adjoint(aderdg_solver *s, const double *weight_dev, double *lam_dev);

/* Gauss-Legendre nodes xi[n] and weights w[n] on [0,1] (the library's basis). */
aderdg_status aderdg_nodes(int n, double *xi, double *w);

/* info[0..7] = n, dim, V, S (= n^dim), F (= n^(dim-1)), Picard iterations,
 * cells (total), bytes per cell that aderdg_copy_faces writes.              */
aderdg_status aderdg_info(const aderdg_solver *s, long long *info);

/* Device pointer of the state (for zero-copy use by the caller; stream-ordered).
 * Errors: UNSUPPORTED while the state is held in a storage format other than
 * FP64 (use aderdg_get_state, which widens it).                              */
aderdg_status aderdg_state_ptr(aderdg_solver *s, double **dev_ptr);

/* Kernel timing: when enabled, every launch of aderdg_step is bracketed by
 * HIP events on the solver's stream.  aderdg_step runs the predictor of its
 * first step, one fused launch per later step (the corrector of the previous
 * step and the predictor of this one) and the corrector of its last step.
 * aderdg_get_timing synchronises and returns out[0] = total ms of the
 * separate predictor launches, out[1] = of the separate corrector launches,
 * out[2] = number of steps timed, out[3] = total ms of the fused launches,
 * out[4] = number of fused launches; then resets.                           */
aderdg_status aderdg_set_timing(aderdg_solver *s, int enable);
aderdg_status aderdg_get_timing(aderdg_solver *s, double *out);

/* Per-handle description of the last error ("" if none).                    */
const char *aderdg_last_error(const aderdg_solver *s);

#ifdef __cplusplus
}
#endif
#endif
