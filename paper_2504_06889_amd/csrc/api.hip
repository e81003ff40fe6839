// C ABI of the ADER-DG library (declared in include/aderdg.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "aderdg.h"
#include "adjoint.h"
#include "basis.h"
#include "registry.h"

using namespace aderdg;

// ---------------------------------------------------------------------------
// Kernel registry
// ---------------------------------------------------------------------------
namespace aderdg {
static std::map<std::tuple<int, int, int>, KernelSet> &registry() {
    static std::map<std::tuple<int, int, int>, KernelSet> r;
    return r;
}
void register_kernels(int pde, int dim, int order, const KernelSet &ks) {
    registry()[std::make_tuple(pde, dim, order)] = ks;
}
const KernelSet *find_kernels(int pde, int dim, int order) {
    auto it = registry().find(std::make_tuple(pde, dim, order));
    return it == registry().end() ? nullptr : &it->second;
}
}  // namespace aderdg

// ---------------------------------------------------------------------------
// Small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(unsigned long long *p, unsigned long long v) { *p = v; }
__global__ void k_fill_i32(int *p, int v) { *p = v; }
// Convert a state between storage precisions (FP64 in or out, or both in the
// held format): dst[i] = src[i] rounded to the destination format.
__global__ __launch_bounds__(256) void k_convert_state(const void *src, int sp_src, void *dst, int sp_dst, long n) {
    for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256)
        store_state(dst, i, load_state(src, i, sp_src), sp_dst);
}

// dst[r][k] = src[r][k] for the first of the two halves of every row:
// rows of 2 * hw doubles in, hw doubles out.
__global__ __launch_bounds__(256) void k_copy_first_halves(double *dst, const double *src, long hw, long n) {
    for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const long r = i / hw;
        dst[i] = src[i + r * hw];
    }
}

// -sigma times the time operator, its row sums and weighted column sums
// (one 64-thread block; kMaxN^2 = 64).
__global__ __launch_bounds__(64) void k_scale_time(const DevBasis *B, double sigma, ScaledTime *o) {
    const int i = threadIdx.x, r = i / kMaxN, c = i % kMaxN;
    o->At[r][c] = -sigma * B->Atau[r][c];
    if (i < kMaxN) {
        o->Arow[i] = -sigma * B->Arow[i];
        o->wA[i] = -sigma * B->wA[i];
    }
}

__global__ __launch_bounds__(256) void k_nonfinite(const void *x, int sp, long n, int *flag) {
    int bad = 0;
    for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256)
        bad |= !isfinite(load_state(x, i, sp));
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0 && bad) atomicOr(flag, 1);
}

// p_h(x_r) = sum_s prod_j phi[r][j][i_j(s)] Q[cell_r][0][s]
__global__ void k_receivers(const void *Q, int sp, int V, int S, int n, int dim, int nrec, const long *rcell,
                            const double *rphi, double *out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrec) return;
    const long q0 = rcell[r] * V * S;
    const double *ph = rphi + (long)r * 3 * kMaxN;
    double acc = 0.0;
    for (int s = 0; s < S; s++) {
        double w = ph[s % n];
        if (dim > 1) w *= ph[kMaxN + (s / n) % n];
        if (dim > 2) w *= ph[2 * kMaxN + s / (n * n)];
        acc += w * load_state(Q, q0 + s, sp);
    }
    out[r] = acc;
}

// ---------------------------------------------------------------------------
// Solver object
// ---------------------------------------------------------------------------
struct aderdg_solver {
    aderdg_config cfg;
    int n, d, V, S, F, iters;
    long ncell;
    double h, t = 0.0;
    hipStream_t stream;
    const KernelSet *ks;
    DevBasis hB;
    DevBasis *dB = nullptr;
    ScaledTime *dST = nullptr;  // time operator scaled for the dt of the last step call
    void *dQ = nullptr;         // state in the storage precision prec[ADERDG_K_STORAGE]
    void *dFaces = nullptr;     // face data of the last predictor
    void *dFaces2 = nullptr;    // second buffer: a fused step reads one and writes the other
    size_t face_elems = 0;
    double *dMat = nullptr;
    double *dSrcPhi = nullptr;
    long src_cell = -1;
    double src_f0 = 0, src_t0 = 0, src_amp = 0;
    int nrec = 0;
    long *dRecCell = nullptr;
    double *dRecPhi = nullptr;
    // receivers grouped by cell (for the deterministic adjoint scatter)
    int nrec_cells = 0;
    long *dRecUcell = nullptr;
    int *dRecStart = nullptr, *dRecOrder = nullptr;
    unsigned long long *dScalar = nullptr;
    int *dFlag = nullptr;
    int prec[4] = {0, 0, 0, 0};
    int predictor = ADERDG_PICARD;
    int device = -1;  // HIP device current at creation
    AdjointWork adj;
    bool timing = false;
    std::vector<hipEvent_t> ev;  // 2 events per timed launch
    std::vector<int> ev_kind;    // 0 predictor, 1 corrector, 2 fused corrector + predictor
    int ev_used = 0, steps_timed = 0;
    std::string err;
};

#define FAIL(s, code, ...)                                                   \
    do {                                                                     \
        char _b[512];                                                        \
        snprintf(_b, sizeof(_b), __VA_ARGS__);                               \
        (s)->err = _b;                                                       \
        return code;                                                         \
    } while (0)

#define HIPC(s, call)                                                                      \
    do {                                                                                   \
        hipError_t _e = (call);                                                            \
        if (_e != hipSuccess) FAIL(s, ADERDG_E_DEVICE, "%s: %s", #call, hipGetErrorString(_e)); \
    } while (0)

static thread_local std::string g_create_err;

static void free_all(aderdg_solver *s) {
    for (auto e : s->ev) hipEventDestroy(e);
    s->ev.clear();
    hipFree(s->dB);
    hipFree(s->dST);
    hipFree(s->dQ);
    hipFree(s->dFaces);
    hipFree(s->dFaces2);
    hipFree(s->dMat);
    hipFree(s->dSrcPhi);
    hipFree(s->dRecCell);
    hipFree(s->dRecPhi);
    hipFree(s->dRecUcell);
    hipFree(s->dRecStart);
    hipFree(s->dRecOrder);
    hipFree(s->dScalar);
    hipFree(s->dFlag);
    adjoint_free(s->adj);
}

static long state_elems(const aderdg_solver *s) { return s->ncell * (long)s->V * s->S; }

static int nvars(int pde, int dim) {
    switch (pde) {
    case ADERDG_ACOUSTIC: return 1 + dim;
    case ADERDG_ELASTIC: return dim * (dim + 1) / 2 + dim;
    case ADERDG_EULER: return 2 + dim;
    case ADERDG_SWE: return dim == 2 ? 4 : -1;
    }
    return -1;
}

extern "C" {

aderdg_status aderdg_create(const aderdg_config *cfg, void *hip_stream, aderdg_solver **out) {
    if (!cfg || !out) return ADERDG_E_INVALID;
    *out = nullptr;
    auto *s = new aderdg_solver();
    s->cfg = *cfg;
    s->stream = (hipStream_t)hip_stream;
    if (cfg->dim < 2 || cfg->dim > 3) {
        g_create_err = "dim must be 2 or 3";
        delete s;
        return ADERDG_E_INVALID;
    }
    s->d = cfg->dim;
    s->n = cfg->order + 1;
    s->V = nvars(cfg->pde, cfg->dim);
    if (cfg->order < 0 || s->n > kMaxN || s->V < 0) {
        g_create_err = "invalid order or pde/dim";
        delete s;
        return ADERDG_E_INVALID;
    }
    s->S = 1;
    for (int i = 0; i < s->d; i++) s->S *= s->n;
    s->F = s->S / s->n;
    s->iters = cfg->picard_iters > 0 ? cfg->picard_iters : cfg->order + 1;
    s->ncell = 1;
    for (int i = 0; i < s->d; i++) {
        if (cfg->cells[i] < 1) {
            g_create_err = "cells must be positive";
            delete s;
            return ADERDG_E_INVALID;
        }
        s->ncell *= cfg->cells[i];
    }
    if (s->ncell > 2147483647L) {
        g_create_err = "at most 2^31 - 1 cells";
        delete s;
        return ADERDG_E_INVALID;
    }
    s->h = (cfg->hi[0] - cfg->lo[0]) / cfg->cells[0];
    for (int i = 0; i < s->d; i++) {
        const double hi = (cfg->hi[i] - cfg->lo[i]) / cfg->cells[i];
        if (!(hi > 0) || std::fabs(hi - s->h) > 1e-12 * s->h) {
            g_create_err = "cells must be cubes with positive size";
            delete s;
            return ADERDG_E_INVALID;
        }
    }
    s->ks = find_kernels(cfg->pde, cfg->dim, cfg->order);
    if (!s->ks) {
        g_create_err = "no kernels built for this (pde, dim, order)";
        delete s;
        return ADERDG_E_UNSUPPORTED;
    }
    if (!build_basis(s->n, s->hB)) {
        g_create_err = "basis construction failed";
        delete s;
        return ADERDG_E_INVALID;
    }
    s->face_elems = (size_t)s->ncell * s->d * 2 * 2 * s->V * s->F;
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        g_create_err = std::string("hipGetDevice: ") + hipGetErrorString(e);
        delete s;
        return ADERDG_E_DEVICE;
    }
    {
        // address of the static scratch array on this device (once per device)
        std::string msg;
        if (noalloc_scratch_init(msg) != 0) {
            g_create_err = msg;
            delete s;
            return ADERDG_E_DEVICE;
        }
    }
    e = hipMalloc(&s->dB, sizeof(DevBasis));
    if (e == hipSuccess) e = hipMalloc(&s->dST, sizeof(ScaledTime));
    if (e == hipSuccess) e = hipMalloc(&s->dQ, sizeof(double) * state_elems(s));
    if (e == hipSuccess) e = hipMalloc(&s->dFaces, sizeof(double) * s->face_elems);
    if (e == hipSuccess) e = hipMalloc(&s->dFaces2, sizeof(double) * s->face_elems);
    if (e == hipSuccess) e = hipMalloc(&s->dScalar, sizeof(unsigned long long) * 4);
    if (e == hipSuccess) e = hipMalloc(&s->dFlag, sizeof(int) * 4);
    if (e != hipSuccess) {
        g_create_err = std::string("device allocation failed: ") + hipGetErrorString(e);
        free_all(s);
        delete s;
        return ADERDG_E_OOM;
    }
    e = hipMemcpy(s->dB, &s->hB, sizeof(DevBasis), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemsetAsync(s->dQ, 0, sizeof(double) * state_elems(s), s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->dFlag, 0, sizeof(int) * 4, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        g_create_err = std::string("device initialisation failed: ") + hipGetErrorString(e);
        free_all(s);
        delete s;
        return ADERDG_E_DEVICE;
    }
    *out = s;
    return ADERDG_OK;
}

aderdg_status aderdg_destroy(aderdg_solver *s) {
    if (!s) return ADERDG_OK;
    hipStreamSynchronize(s->stream);
    free_all(s);
    delete s;
    return ADERDG_OK;
}

static long grid256(long n) {
    const long g = (n + 255) / 256;
    return g < 8192 ? g : 8192;
}

static int storage(const aderdg_solver *s) { return s->prec[ADERDG_K_STORAGE]; }

// FP64 staging for host copies of a narrow state: the second face buffer (its
// contents are only read by the fused launches inside one aderdg_step call,
// and it holds at least a state's doubles: 4d/n >= 1 for n <= 8).
static void *staging(aderdg_solver *s) { return s->dFaces2; }

static void convert_state(aderdg_solver *s, const void *src, int sp_src, void *dst, int sp_dst) {
    hipLaunchKernelGGL(k_convert_state, dim3(grid256(state_elems(s))), dim3(256), 0, s->stream, src, sp_src, dst,
                       sp_dst, state_elems(s));
}

aderdg_status aderdg_set_state(aderdg_solver *s, const double *Q, int is_device) {
    if (!s) return ADERDG_E_INVALID;
    if (!Q) FAIL(s, ADERDG_E_INVALID, "null state pointer");
    const size_t bytes = sizeof(double) * state_elems(s);
    if (storage(s) == ADERDG_FP64) {
        HIPC(s, hipMemcpyAsync(s->dQ, Q, bytes, is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                               s->stream));
    } else if (is_device) {
        convert_state(s, Q, ADERDG_FP64, s->dQ, storage(s));
    } else {
        HIPC(s, hipMemcpyAsync(staging(s), Q, bytes, hipMemcpyHostToDevice, s->stream));
        convert_state(s, staging(s), ADERDG_FP64, s->dQ, storage(s));
    }
    HIPC(s, hipGetLastError());
    if (!is_device) HIPC(s, hipStreamSynchronize(s->stream));
    return ADERDG_OK;
}
static aderdg_status check_finite(aderdg_solver *s, const void *x, int sp, long count, bool *ok) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, s->stream, s->dFlag, 0);
    long g = (count + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_nonfinite, dim3(g), dim3(256), 0, s->stream, x, sp, count, s->dFlag);
    int flag = 0;
    HIPC(s, hipMemcpyAsync(&flag, s->dFlag, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIPC(s, hipStreamSynchronize(s->stream));
    *ok = flag == 0;
    return ADERDG_OK;
}

aderdg_status aderdg_get_state(aderdg_solver *s, double *Q, int is_device) {
    if (!s) return ADERDG_E_INVALID;
    if (!Q) FAIL(s, ADERDG_E_INVALID, "null state pointer");
    const size_t bytes = sizeof(double) * state_elems(s);
    if (storage(s) == ADERDG_FP64) {
        HIPC(s, hipMemcpyAsync(Q, s->dQ, bytes, is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                               s->stream));
    } else if (is_device) {
        convert_state(s, s->dQ, storage(s), Q, ADERDG_FP64);
    } else {
        convert_state(s, s->dQ, storage(s), staging(s), ADERDG_FP64);
        HIPC(s, hipMemcpyAsync(Q, staging(s), bytes, hipMemcpyDeviceToHost, s->stream));
    }
    bool ok = true;
    aderdg_status st = check_finite(s, s->dQ, storage(s), state_elems(s), &ok);
    if (st != ADERDG_OK) return st;
    if (!ok) FAIL(s, ADERDG_E_NONFINITE, "state holds NaN or Inf");
    return ADERDG_OK;
}

aderdg_status aderdg_set_material(aderdg_solver *s, const double *c, int is_device) {
    if (!s) return ADERDG_E_INVALID;
    if (!c) FAIL(s, ADERDG_E_INVALID, "null material pointer");
    if (s->cfg.pde != ADERDG_ACOUSTIC) FAIL(s, ADERDG_E_UNSUPPORTED, "per-cell material is for acoustics only");
    if (!s->dMat) HIPC(s, hipMalloc(&s->dMat, sizeof(double) * s->ncell));
    HIPC(s, hipMemcpyAsync(s->dMat, c, sizeof(double) * s->ncell,
                           is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->stream));
    if (!is_device) HIPC(s, hipStreamSynchronize(s->stream));
    return ADERDG_OK;
}

aderdg_status aderdg_set_predictor(aderdg_solver *s, int kind) {
    if (!s) return ADERDG_E_INVALID;
    if (kind != ADERDG_PICARD && kind != ADERDG_CK) FAIL(s, ADERDG_E_INVALID, "unknown predictor %d", kind);
    if (kind == ADERDG_CK) {
        if (s->cfg.pde != ADERDG_ACOUSTIC && s->cfg.pde != ADERDG_ELASTIC)
            FAIL(s, ADERDG_E_UNSUPPORTED, "the Cauchy-Kowalevskaya predictor needs a linear PDE");
        if (s->src_cell >= 0) FAIL(s, ADERDG_E_UNSUPPORTED, "the Cauchy-Kowalevskaya predictor takes no point source");
    }
    s->predictor = kind;
    return ADERDG_OK;
}

aderdg_status aderdg_set_precision(aderdg_solver *s, int kernel, int prec) {
    if (!s) return ADERDG_E_INVALID;
    if (kernel < 0 || kernel > 3 || prec < 0 || prec > 3) FAIL(s, ADERDG_E_INVALID, "unknown kernel or precision");
    if (kernel == ADERDG_K_STORAGE) {
        // the held state moves to a buffer of the new format, each value rounded
        // to it (through FP64 staging)
        const int old = storage(s);
        if (prec == old) return ADERDG_OK;
        void *nq = nullptr;
        HIPC(s, hipStreamSynchronize(s->stream));
        if (hipMalloc(&nq, (size_t)state_bytes(prec) * state_elems(s)) != hipSuccess)
            FAIL(s, ADERDG_E_OOM, "state allocation failed");
        convert_state(s, s->dQ, old, staging(s), ADERDG_FP64);
        convert_state(s, staging(s), ADERDG_FP64, nq, prec);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) {
            hipFree(nq);
            FAIL(s, ADERDG_E_DEVICE, "state conversion: %s", hipGetErrorString(e));
        }
        hipFree(s->dQ);
        s->dQ = nq;
        s->prec[kernel] = prec;
        return ADERDG_OK;
    }
    if (kernel == ADERDG_K_PREDICTOR && !s->ks->pred[prec])
        FAIL(s, ADERDG_E_UNSUPPORTED, "predictor precision %d not built for this (pde, dim, order)", prec);
    s->prec[kernel] = prec;
    return ADERDG_OK;
}

static PdeArgs pde_args(const aderdg_solver *s) {
    PdeArgs p;
    for (int i = 0; i < 8; i++) p.prm[i] = s->cfg.params[i];
    p.mat = s->dMat;
    return p;
}

aderdg_status aderdg_max_dt(aderdg_solver *s, double cfl, double *dt_out) {
    if (!s || !dt_out) return ADERDG_E_INVALID;
    if (!(cfl > 0)) FAIL(s, ADERDG_E_INVALID, "cfl must be positive");
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s->stream, s->dScalar, 0ull);
    s->ks->maxeig(s->dQ, storage(s), pde_args(s), s->ncell, s->dScalar, s->stream);
    unsigned long long bits = 0;
    HIPC(s, hipMemcpyAsync(&bits, s->dScalar, sizeof(bits), hipMemcpyDeviceToHost, s->stream));
    HIPC(s, hipStreamSynchronize(s->stream));
    double lmax;
    std::memcpy(&lmax, &bits, sizeof(double));
    if (!(lmax > 0) || !std::isfinite(lmax)) FAIL(s, ADERDG_E_NONFINITE, "maximum wave speed is %g", lmax);
    *dt_out = cfl * s->h / (s->d * (2.0 * s->cfg.order + 1.0) * lmax);
    return ADERDG_OK;
}

// The point source's time function (Ricker wavelet) at the n time nodes of the
// step [t, t + dt], times h, and its time average (zero without a source).
static double ricker_host(double t, double f0, double t0, double amp) {
    const double x = M_PI * f0 * (t - t0), q = x * x;
    return amp * (1.0 - 2.0 * q) * std::exp(-q);
}
static void source_values(const aderdg_solver *s, double t, double dt, double *src_s, double *src_bar) {
    *src_bar = 0.0;
    for (int b = 0; b < kMaxN; b++) src_s[b] = 0.0;
    if (s->src_cell < 0) return;
    for (int b = 0; b < s->n; b++) {
        const double r = ricker_host(t + s->hB.xi[b] * dt, s->src_f0, s->src_t0, s->src_amp);
        src_s[b] = s->h * r;
        *src_bar += s->hB.w[b] * r;
    }
}

// Form the scaled time operator for step size dt on the solver's stream,
// ahead of the launches that read it (every call, so that captured work
// replays with its own dt).
static aderdg_status scale_time(aderdg_solver *s, double dt) {
    hipLaunchKernelGGL(k_scale_time, dim3(1), dim3(kMaxN * kMaxN), 0, s->stream, (const DevBasis *)s->dB, dt / s->h,
                       s->dST);
    HIPC(s, hipGetLastError());
    return ADERDG_OK;
}

static StepArgs step_args(aderdg_solver *s, double dt, double t) {
    StepArgs a{};
    a.Q = s->dQ;
    a.faces = s->dFaces;
    a.faces_in = nullptr;
    a.B = s->dB;
    a.st = s->dST;
    a.pde = pde_args(s);
    a.ncell = s->ncell;
    for (int i = 0; i < 3; i++) a.cells[i] = i < s->d ? s->cfg.cells[i] : 1;
    a.dt = dt;
    a.inv_h = 1.0 / s->h;
    a.sigma = dt / s->h;
    a.t = t;
    a.h = s->h;
    a.vol_prec = s->prec[ADERDG_K_VOLUME];
    a.flux_prec = s->prec[ADERDG_K_FLUX];
    a.iters = s->iters;
    a.ck = s->predictor == ADERDG_CK;
    a.store_prec = s->prec[ADERDG_K_STORAGE];
    a.write_state = 1;
    a.src_cell = s->src_cell;
    a.src_phi = s->dSrcPhi;
    source_values(s, t, dt, a.src_s, &a.src_bar);
    return a;
}

// Launch with optional timing events (kind: 0 predictor, 1 corrector, 2 fused).
static aderdg_status launch(aderdg_solver *s, StepFn fn, const StepArgs &a, int kind) {
    if (!s->timing) {
        fn(a, s->stream);
        return ADERDG_OK;
    }
    if ((size_t)(s->ev_used + 2) > s->ev.size()) {
        for (int i = 0; i < 2 * 64; i++) {
            hipEvent_t x;
            HIPC(s, hipEventCreate(&x));
            s->ev.push_back(x);
            s->ev_kind.push_back(0);
        }
    }
    hipEvent_t *e = &s->ev[s->ev_used];
    s->ev_kind[s->ev_used] = kind;
    s->ev_used += 2;
    HIPC(s, hipEventRecord(e[0], s->stream));
    fn(a, s->stream);
    HIPC(s, hipEventRecord(e[1], s->stream));
    return ADERDG_OK;
}

// nsteps steps of Alg. 1: the predictor of step 1, then for every later step
// one fused launch (corrector of the previous step, kept in registers, and
// the predictor of this step; the face data alternate between two buffers),
// and the corrector of the last step.  Identical arithmetic to separate
// predictor and corrector launches.
aderdg_status aderdg_step(aderdg_solver *s, double dt, int nsteps) {
    if (!s) return ADERDG_E_INVALID;
    if (!(dt > 0) || nsteps < 0) FAIL(s, ADERDG_E_INVALID, "dt must be positive and nsteps >= 0");
    if (nsteps == 0) return ADERDG_OK;
    const StepFn pred = s->ks->pred[s->prec[ADERDG_K_PREDICTOR]];
    const StepFn fused = s->ks->fused[s->prec[ADERDG_K_PREDICTOR]];
    const StepFn corr = s->ks->corr[s->prec[ADERDG_K_FLUX]];
    aderdg_status rc;
    if ((rc = scale_time(s, dt)) != ADERDG_OK) return rc;
    StepArgs a = step_args(s, dt, s->t);
    if ((rc = launch(s, pred, a, 0)) != ADERDG_OK) return rc;
    for (int k = 1; k < nsteps; k++) {
        std::swap(s->dFaces, s->dFaces2);
        a = step_args(s, dt, s->t + k * dt);
        a.faces_in = s->dFaces2;
        if ((rc = launch(s, fused, a, 2)) != ADERDG_OK) return rc;
    }
    a = step_args(s, dt, s->t + (nsteps - 1) * dt);
    if ((rc = launch(s, corr, a, 1)) != ADERDG_OK) return rc;
    HIPC(s, hipGetLastError());
    if (s->timing) s->steps_timed += nsteps;
    s->t += nsteps * dt;
    return ADERDG_OK;
}

aderdg_status aderdg_set_timing(aderdg_solver *s, int enable) {
    if (!s) return ADERDG_E_INVALID;
    s->timing = enable != 0;
    s->ev_used = 0;
    s->steps_timed = 0;
    return ADERDG_OK;
}

aderdg_status aderdg_get_timing(aderdg_solver *s, double *out) {
    if (!s || !out) return ADERDG_E_INVALID;
    HIPC(s, hipStreamSynchronize(s->stream));
    double ms[3] = {0.0, 0.0, 0.0};
    int cnt[3] = {0, 0, 0};
    for (int i = 0; i + 1 < s->ev_used; i += 2) {
        float x = 0.f;
        HIPC(s, hipEventElapsedTime(&x, s->ev[i], s->ev[i + 1]));
        ms[s->ev_kind[i]] += x;
        cnt[s->ev_kind[i]]++;
    }
    out[0] = ms[0];
    out[1] = ms[1];
    out[2] = s->steps_timed;
    out[3] = ms[2];
    out[4] = cnt[2];
    s->ev_used = 0;
    s->steps_timed = 0;
    return ADERDG_OK;
}

aderdg_status aderdg_set_time(aderdg_solver *s, double t) {
    if (!s) return ADERDG_E_INVALID;
    s->t = t;
    return ADERDG_OK;
}

aderdg_status aderdg_get_time(const aderdg_solver *s, double *t) {
    if (!s || !t) return ADERDG_E_INVALID;
    *t = s->t;
    return ADERDG_OK;
}

// Locate x: cell index and local coordinates in [0,1]^d.
static bool locate(const aderdg_solver *s, const double *x, long *cell, double *loc) {
    long c = 0, m = 1;
    for (int i = 0; i < s->d; i++) {
        const double u = (x[i] - s->cfg.lo[i]) / s->h;
        long ci = (long)std::floor(u);
        if (ci == s->cfg.cells[i] && u <= s->cfg.cells[i] + 1e-12) ci = s->cfg.cells[i] - 1;
        if (ci < 0 || ci >= s->cfg.cells[i]) return false;
        loc[i] = u - ci;
        c += ci * m;
        m *= s->cfg.cells[i];
    }
    *cell = c;
    return true;
}

aderdg_status aderdg_set_source(aderdg_solver *s, const double x[3], double f0, double t0, double amp) {
    if (!s || !x) return ADERDG_E_INVALID;
    if (s->cfg.pde != ADERDG_ACOUSTIC) FAIL(s, ADERDG_E_UNSUPPORTED, "point sources are for acoustics only");
    if (s->predictor != ADERDG_PICARD)
        FAIL(s, ADERDG_E_UNSUPPORTED, "point sources need the Picard predictor");
    long cell;
    double loc[3];
    if (!locate(s, x, &cell, loc)) FAIL(s, ADERDG_E_INVALID, "source outside the domain");
    std::vector<double> phi(s->S);
    const double hd = std::pow(s->h, s->d);
    for (int sn = 0; sn < s->S; sn++) {
        double p = 1.0, W = 1.0;
        int r = sn;
        for (int i = 0; i < s->d; i++) {
            const int k = r % s->n;
            r /= s->n;
            p *= lagrange_value(s->n, s->hB.xi, k, loc[i]);
            W *= s->hB.w[k];
        }
        phi[sn] = p / (hd * W);
    }
    if (!s->dSrcPhi) HIPC(s, hipMalloc(&s->dSrcPhi, sizeof(double) * s->S));
    HIPC(s, hipMemcpy(s->dSrcPhi, phi.data(), sizeof(double) * s->S, hipMemcpyHostToDevice));
    s->src_cell = cell;
    s->src_f0 = f0;
    s->src_t0 = t0;
    s->src_amp = amp;
    return ADERDG_OK;
}

aderdg_status aderdg_set_receivers(aderdg_solver *s, int nrec, const double *xyz) {
    if (!s || nrec < 0 || (nrec > 0 && !xyz)) return ADERDG_E_INVALID;
    std::vector<long> cells(nrec);
    std::vector<double> phi((size_t)nrec * 3 * kMaxN, 0.0);
    for (int r = 0; r < nrec; r++) {
        double loc[3];
        if (!locate(s, xyz + 3 * r, &cells[r], loc)) FAIL(s, ADERDG_E_INVALID, "receiver %d outside the domain", r);
        for (int i = 0; i < s->d; i++)
            for (int k = 0; k < s->n; k++)
                phi[(size_t)r * 3 * kMaxN + i * kMaxN + k] = lagrange_value(s->n, s->hB.xi, k, loc[i]);
    }
    // receivers grouped by cell: the adjoint scatter sums each cell's receivers
    // in this fixed order
    std::vector<int> order(nrec);
    for (int r = 0; r < nrec; r++) order[r] = r;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cells[a] < cells[b]; });
    std::vector<long> ucell;
    std::vector<int> start;
    for (int k = 0; k < nrec; k++) {
        if (k == 0 || cells[order[k]] != cells[order[k - 1]]) {
            ucell.push_back(cells[order[k]]);
            start.push_back(k);
        }
    }
    start.push_back(nrec);
    hipFree(s->dRecCell);
    hipFree(s->dRecPhi);
    hipFree(s->dRecUcell);
    hipFree(s->dRecStart);
    hipFree(s->dRecOrder);
    s->dRecCell = nullptr;
    s->dRecPhi = nullptr;
    s->dRecUcell = nullptr;
    s->dRecStart = s->dRecOrder = nullptr;
    s->nrec = nrec;
    s->nrec_cells = (int)ucell.size();
    if (nrec == 0) return ADERDG_OK;
    HIPC(s, hipMalloc(&s->dRecCell, sizeof(long) * nrec));
    HIPC(s, hipMalloc(&s->dRecPhi, sizeof(double) * phi.size()));
    HIPC(s, hipMalloc(&s->dRecUcell, sizeof(long) * ucell.size()));
    HIPC(s, hipMalloc(&s->dRecStart, sizeof(int) * start.size()));
    HIPC(s, hipMalloc(&s->dRecOrder, sizeof(int) * nrec));
    HIPC(s, hipMemcpy(s->dRecCell, cells.data(), sizeof(long) * nrec, hipMemcpyHostToDevice));
    HIPC(s, hipMemcpy(s->dRecPhi, phi.data(), sizeof(double) * phi.size(), hipMemcpyHostToDevice));
    HIPC(s, hipMemcpy(s->dRecUcell, ucell.data(), sizeof(long) * ucell.size(), hipMemcpyHostToDevice));
    HIPC(s, hipMemcpy(s->dRecStart, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice));
    HIPC(s, hipMemcpy(s->dRecOrder, order.data(), sizeof(int) * nrec, hipMemcpyHostToDevice));
    return ADERDG_OK;
}

aderdg_status aderdg_read_receivers(aderdg_solver *s, double *out, int is_device) {
    if (!s || !out) return ADERDG_E_INVALID;
    if (s->nrec == 0) return ADERDG_OK;
    double *dst = out;
    double *tmp = nullptr;
    if (!is_device) {
        HIPC(s, hipMalloc(&tmp, sizeof(double) * s->nrec));
        dst = tmp;
    }
    hipLaunchKernelGGL(k_receivers, dim3((s->nrec + 63) / 64), dim3(64), 0, s->stream, s->dQ, storage(s), s->V,
                       s->S, s->n,
                       s->d, s->nrec, s->dRecCell, s->dRecPhi, dst);
    if (!is_device) {
        hipError_t e = hipMemcpyAsync(out, tmp, sizeof(double) * s->nrec, hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        hipFree(tmp);
        if (e != hipSuccess) FAIL(s, ADERDG_E_DEVICE, "receiver copy: %s", hipGetErrorString(e));
    }
    return ADERDG_OK;
}

static aderdg_status step_adjoint(aderdg_solver *s, double dt, double t, const double *Qn_dev, const void *fwd,
                                  double *lam_dev, double *grad_dev, bool noalloc = false) {
    if (!s || !Qn_dev || !lam_dev || !grad_dev) return ADERDG_E_INVALID;
    if (!(dt > 0)) FAIL(s, ADERDG_E_INVALID, "dt must be positive");
    if (s->cfg.pde != ADERDG_ACOUSTIC || !s->dMat)
        FAIL(s, ADERDG_E_UNSUPPORTED, "the adjoint is built for acoustics with a per-cell material");
    if (s->prec[ADERDG_K_FLUX]) FAIL(s, ADERDG_E_UNSUPPORTED, "the adjoint needs the flux kernel in FP64");
    if ((s->prec[ADERDG_K_PREDICTOR] == ADERDG_FP64) != (s->prec[ADERDG_K_VOLUME] == ADERDG_FP64))
        FAIL(s, ADERDG_E_UNSUPPORTED, "the adjoint needs the predictor and volume kernels both in FP64 or both lower");
    if (s->predictor != ADERDG_PICARD) FAIL(s, ADERDG_E_UNSUPPORTED, "the adjoint differentiates the Picard predictor");
    if (s->prec[ADERDG_K_STORAGE] != ADERDG_FP64) FAIL(s, ADERDG_E_UNSUPPORTED, "the adjoint needs the state in FP64");
    AdjointArgs a{};
    a.pred = s->ks->pred[s->prec[ADERDG_K_PREDICTOR]];
    a.prec_pred = s->prec[ADERDG_K_PREDICTOR];
    a.prec_vol = s->prec[ADERDG_K_VOLUME];
    a.cfg_pde = s->cfg.pde;
    a.dim = s->d;
    a.order = s->cfg.order;
    a.ncell = s->ncell;
    for (int i = 0; i < 3; i++) a.cells[i] = i < s->d ? s->cfg.cells[i] : 1;
    a.B = s->dB;
    a.st = s->dST;
    a.pde = pde_args(s);
    a.dt = dt;
    a.t = t;
    a.inv_h = 1.0 / s->h;
    a.sigma = dt / s->h;
    a.iters = s->iters;
    a.Qn = Qn_dev;
    a.fwdface = fwd;
    a.lam = lam_dev;
    a.grad = grad_dev;
    a.src_cell = s->src_cell;
    a.src_phi = s->dSrcPhi;
    a.src_f0 = s->src_f0;
    a.src_t0 = s->src_t0;
    a.src_amp = s->src_amp;
    source_values(s, t, dt, a.src_s, &a.src_bar);
    std::string msg;
    void *scr = nullptr;
    if (noalloc) {
        scr = noalloc_scratch(s->device);
        if (!scr) FAIL(s, ADERDG_E_DEVICE, "the scratch array is not set up on device %d", s->device);
        const size_t need = adjoint_lamface_bytes(a);
        if (need > kNoAllocScratchBytes)
            FAIL(s, ADERDG_E_INVALID,
                 "the adjoint face restrictions need %zu bytes, more than the %zu-byte scratch array "
                 "(ncell * dim * 2 * (dim + 1) * (order + 1)^(dim - 1) * 8 bytes)",
                 need, (size_t)kNoAllocScratchBytes);
    }
    {  // read by the adjoint's forward sweep and by the predictor that recomputes the face data
        const aderdg_status rs = scale_time(s, dt);
        if (rs != ADERDG_OK) return rs;
    }
    const int rc = adjoint_step(s->adj, a, s->stream, msg, scr);
    if (rc != 0) {
        s->err = msg;
        return (aderdg_status)rc;
    }
    return ADERDG_OK;
}

aderdg_status aderdg_step_adjoint(aderdg_solver *s, double dt, double t, const double *Qn_dev, double *lam_dev,
                                  double *grad_dev) {
    return step_adjoint(s, dt, t, Qn_dev, nullptr, lam_dev, grad_dev);
}

aderdg_status aderdg_step_adjoint_faces(aderdg_solver *s, double dt, double t, const double *Qn_dev,
                                        const void *fwd_faces_dev, double *lam_dev, double *grad_dev) {
    if (!fwd_faces_dev) return ADERDG_E_INVALID;
    return step_adjoint(s, dt, t, Qn_dev, fwd_faces_dev, lam_dev, grad_dev);
}

aderdg_status aderdg_step_adjoint_faces_noalloc(aderdg_solver *s, double dt, double t, const double *Qn_dev,
                                                const void *fwd_faces_dev, double *lam_dev, double *grad_dev) {
    if (!fwd_faces_dev) return ADERDG_E_INVALID;
    return step_adjoint(s, dt, t, Qn_dev, fwd_faces_dev, lam_dev, grad_dev, true);
}

// The predictor leaves the f halves of the face buffer unwritten when the
// corrector evaluates the flux from the projected q: a linear PDE with FP64
// faces.  Copies of the face data then hold the q halves only.
static bool faces_q_only(const aderdg_solver *s) {
    return (s->cfg.pde == ADERDG_ACOUSTIC || s->cfg.pde == ADERDG_ELASTIC) && s->prec[ADERDG_K_FLUX] == ADERDG_FP64;
}

aderdg_status aderdg_copy_faces(aderdg_solver *s, void *dst, int is_device) {
    if (!s || !dst) return ADERDG_E_INVALID;
    const hipMemcpyKind kind = is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const int fp = s->prec[ADERDG_K_FLUX];
    const size_t half = (size_t)s->V * s->F * (fp == 0 ? 8 : (fp == 1 ? 4 : 2));  // one [var][face node] block
    const size_t rows = (size_t)s->ncell * s->d * 2;                                // (cell, dir, side)
    if (faces_q_only(s) && is_device) {  // FP64 halves: whole doubles
        const long hw = (long)(half / sizeof(double)), n = hw * (long)rows;
        hipLaunchKernelGGL(k_copy_first_halves, dim3(grid256(n)), dim3(256), 0, s->stream, (double *)dst,
                           (const double *)s->dFaces, hw, n);
        HIPC(s, hipGetLastError());
    } else if (faces_q_only(s)) {
        HIPC(s, hipMemcpy2DAsync(dst, half, s->dFaces, 2 * half, half, rows, kind, s->stream));
    } else
        HIPC(s, hipMemcpyAsync(dst, s->dFaces, 2 * half * rows, kind, s->stream));
    if (!is_device) HIPC(s, hipStreamSynchronize(s->stream));
    return ADERDG_OK;
}

aderdg_status aderdg_receivers_adjoint(aderdg_solver *s, const double *weight_dev, double *lam_dev) {
    if (!s || !weight_dev || !lam_dev) return ADERDG_E_INVALID;
    if (s->nrec == 0) return ADERDG_OK;
    receivers_adjoint(lam_dev, s->V, s->S, s->n, s->d, s->nrec_cells, s->dRecUcell, s->dRecStart, s->dRecOrder,
                      s->dRecPhi, weight_dev, s->stream);
    HIPC(s, hipGetLastError());
    return ADERDG_OK;
}

aderdg_status aderdg_nodes(int n, double *xi, double *w) {
    if (n < 1 || n > kMaxN || !xi || !w) return ADERDG_E_INVALID;
    gauss_legendre01(n, xi, w);
    return ADERDG_OK;
}

aderdg_status aderdg_info(const aderdg_solver *s, long long *info) {
    if (!s || !info) return ADERDG_E_INVALID;
    info[0] = s->n;
    info[1] = s->d;
    info[2] = s->V;
    info[3] = s->S;
    info[4] = s->F;
    info[5] = s->iters;
    info[6] = s->ncell;
    const int fp = s->prec[ADERDG_K_FLUX];
    info[7] = (long long)(2 * s->d * (faces_q_only(s) ? 1 : 2) * s->V * s->F) * (fp == 0 ? 8 : (fp == 1 ? 4 : 2));
    return ADERDG_OK;
}

aderdg_status aderdg_state_ptr(aderdg_solver *s, double **dev_ptr) {
    if (!s || !dev_ptr) return ADERDG_E_INVALID;
    if (storage(s) != ADERDG_FP64) FAIL(s, ADERDG_E_UNSUPPORTED, "the state is held in a narrower format");
    *dev_ptr = (double *)s->dQ;
    return ADERDG_OK;
}

const char *aderdg_last_error(const aderdg_solver *s) {
    if (!s) return g_create_err.c_str();
    return s->err.c_str();
}

}  // extern "C"
