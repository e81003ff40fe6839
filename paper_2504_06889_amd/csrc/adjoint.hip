// Discrete adjoint of the ADER-DG step (acoustics, per-cell sound speed): host
// dispatch of the three kernels of one adjoint step.
//   1. k_lamface:   face restrictions L0^T lam, L1^T lam of the incoming adjoint;
//   2. k_predictor: the forward step's face data from Qn (state untouched);
//   3. k_adjoint:   per cell, Rusanov/face/volume adjoints, tangent predictor for
//                   the material derivative, transposed Picard iterations; the
//                   FP64 kernel, or the mixed-precision one when the predictor
//                   and volume contractions run in lower formats.
#include <map>
#include <mutex>
#include <utility>

#include "adjoint.h"
#include "adjoint_kernels.h"
#include "aderdg.h"

namespace aderdg {

// lam[cell][0][s] += sum over the receivers r in that cell of
// weight[r] * prod_j phi[r][j][i_j(s)]: one thread per (receiver cell, node),
// the receivers of a cell summed in a fixed order (sorted by cell, then by
// index), so the result does not depend on scheduling (no atomics).
__global__ void k_receivers_adjoint(double *lam, int V, int S, int n, int dim, int ncells, const long *ucell,
                                    const int *start, const int *order, const double *rphi, const double *weight) {
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= (long)ncells * S) return;
    const int m = i / S, s = i % S;
    double acc = 0.0;
    for (int k = start[m]; k < start[m + 1]; k++) {
        const int r = order[k];
        const double *ph = rphi + (long)r * 3 * kMaxN;
        double w = ph[s % n];
        if (dim > 1) w *= ph[kMaxN + (s / n) % n];
        if (dim > 2) w *= ph[2 * kMaxN + s / (n * n)];
        acc = fma(weight[r], w, acc);
    }
    lam[ucell[m] * V * S + s] += acc;
}

void receivers_adjoint(double *lam, int V, int S, int n, int dim, int ncells, const long *ucell, const int *start,
                       const int *order, const double *rphi, const double *weight, hipStream_t st) {
    const long total = (long)ncells * S;
    hipLaunchKernelGGL(k_receivers_adjoint, dim3((total + 255) / 256), dim3(256), 0, st, lam, V, S, n, dim, ncells,
                       ucell, start, order, rphi, weight);
}

using LamFaceFn = void (*)(const double *, double *, long, const DevBasis *, hipStream_t);
using AdjFn = void (*)(const AdjKArgs &, hipStream_t);

template <int DIM, int N, int PP = P64>
struct AdjInstance {
    static void lamface(const double *lam, double *out, long ncell, const DevBasis *B, hipStream_t st) {
        constexpr int LCB = LamFaceShape<DIM, N>::LCB;
        hipLaunchKernelGGL((k_lamface<DIM, N>), dim3((ncell + LCB - 1) / LCB), dim3(256), 0, st, lam, out, ncell,
                           B);
    }
    static void adjoint(const AdjKArgs &a, hipStream_t st) {
        using Sh = Shape<DIM, N>;
        hipLaunchKernelGGL((k_adjoint<DIM, N, PP>), dim3((a.ncell + Sh::CPB - 1) / Sh::CPB), dim3(Sh::TPB), 0, st,
                           a);
    }
};

struct AdjFns {
    LamFaceFn lamface;
    AdjFn by_prec[4];  // by predictor format; null where no mixed forward predictor is built
};

template <int DIM, int N>
static AdjFns fp64_only() {
    return {&AdjInstance<DIM, N>::lamface, {&AdjInstance<DIM, N>::adjoint, nullptr, nullptr, nullptr}};
}
template <int DIM, int N>
static AdjFns all_formats() {
    return {&AdjInstance<DIM, N>::lamface,
            {&AdjInstance<DIM, N>::adjoint, &AdjInstance<DIM, N, P32>::adjoint, &AdjInstance<DIM, N, PBF16>::adjoint,
             &AdjInstance<DIM, N, PF16>::adjoint}};
}

static const std::map<std::pair<int, int>, AdjFns> &adj_table() {
    static const std::map<std::pair<int, int>, AdjFns> t = {
        {{2, 1}, fp64_only<2, 1>()},   {{2, 2}, fp64_only<2, 2>()},   {{2, 3}, all_formats<2, 3>()},
        {{3, 1}, fp64_only<3, 1>()},   {{3, 2}, all_formats<3, 2>()}, {{3, 5}, all_formats<3, 5>()},
    };
    return t;
}

// Scratch for aderdg_step_adjoint_faces_noalloc: a file-scope device array,
// one copy per GPU at its own address, held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in); it uses the address hipGetSymbolAddress returned on that device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_dev[64];  // resolved address per device id

int noalloc_scratch_init(std::string &msg) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        msg = "no current HIP device for the scratch array";
        return ADERDG_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[dev]) return 0;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return ADERDG_E_DEVICE;
    }
    g_scratch_dev[dev] = p;
    return 0;
}

void *noalloc_scratch(int device) {
    if (device < 0 || device >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_dev[device];
}

size_t adjoint_lamface_bytes(const AdjointArgs &a) {
    const int V = 1 + a.dim;
    size_t F = 1;
    for (int i = 1; i < a.dim; i++) F *= a.order + 1;
    return sizeof(double) * (size_t)a.ncell * a.dim * 2 * V * F;
}

static int ensure(void **p, size_t *have, size_t need) {
    if (*have >= need) return 0;
    hipFree(*p);
    *p = nullptr;
    *have = 0;
    if (hipMalloc(p, need) != hipSuccess) return -1;
    *have = need;
    return 0;
}

int adjoint_step(AdjointWork &w, const AdjointArgs &a, hipStream_t st, std::string &msg, void *lamface_scratch) {
    auto it = adj_table().find(std::make_pair(a.dim, a.order));
    if (it == adj_table().end() || !a.pred) {
        msg = "adjoint not built for this (dim, order)";
        return ADERDG_E_UNSUPPORTED;
    }
    const AdjFn adj = (a.prec_pred >= P64 && a.prec_pred <= PF16) ? it->second.by_prec[a.prec_pred] : nullptr;
    if (!adj) {
        msg = "mixed-precision adjoint not built for this (dim, order)";
        return ADERDG_E_UNSUPPORTED;
    }
    const size_t lf = adjoint_lamface_bytes(a);
    void *lamface = lamface_scratch;
    if (lamface) {
        if (!a.fwdface) {
            msg = "the scratch path needs the forward face data";
            return ADERDG_E_INVALID;
        }
    } else {
        if (ensure(&w.lamface, &w.bytes_lamface, lf) ||
            (!a.fwdface && ensure(&w.fwdface, &w.bytes_fwdface, 2 * lf))) {
            msg = "adjoint work allocation failed";
            return ADERDG_E_OOM;
        }
        lamface = w.lamface;
    }
    // 1. face restrictions of the incoming adjoint
    it->second.lamface(a.lam, (double *)lamface, a.ncell, a.B, st);
    // 2. forward face data of this step (unless the caller kept them)
    const void *fwd = a.fwdface ? a.fwdface : w.fwdface;
    if (!a.fwdface) {
        StepArgs f{};  // zero: Picard predictor, no fused input
        f.Q = const_cast<double *>(a.Qn);
        f.faces = w.fwdface;
        f.B = a.B;
        f.st = a.st;
        f.pde = a.pde;
        f.ncell = a.ncell;
        for (int i = 0; i < 3; i++) f.cells[i] = a.cells[i];
        f.dt = a.dt;
        f.inv_h = a.inv_h;
        f.sigma = a.sigma;
        f.t = a.t;
        f.h = 1.0 / a.inv_h;
        f.vol_prec = a.prec_vol;
        f.flux_prec = 0;
        f.iters = a.iters;
        f.write_state = 0;
        f.src_cell = a.src_cell;
        f.src_phi = a.src_phi;
        for (int b = 0; b < kMaxN; b++) f.src_s[b] = a.src_s[b];
        f.src_bar = a.src_bar;
        a.pred(f, st);
    }
    // 3. the adjoint proper
    AdjKArgs k;
    k.Qn = a.Qn;
    k.lam = a.lam;
    k.grad = a.grad;
    k.lamface = (const double *)lamface;
    k.fwdface = (const double *)fwd;
    // the predictor's own buffer holds both halves; a caller's copy holds the q
    // halves only (aderdg_copy_faces of a linear PDE with FP64 faces)
    k.fwd_halves = a.fwdface ? 1 : 2;
    k.B = a.B;
    k.st = a.st;
    k.pde = a.pde;
    k.ncell = a.ncell;
    for (int i = 0; i < 3; i++) k.cells[i] = a.cells[i];
    k.dt = a.dt;
    k.inv_h = a.inv_h;
    k.sigma = a.sigma;
    k.t = a.t;
    k.iters = a.iters;
    k.src_cell = a.src_cell;
    k.src_phi = a.src_phi;
    for (int b = 0; b < kMaxN; b++) k.src_s[b] = a.src_s[b];
    k.pv = a.prec_vol;
    adj(k, st);
    if (hipGetLastError() != hipSuccess) {
        msg = "adjoint kernel launch failed";
        return ADERDG_E_DEVICE;
    }
    return 0;
}

void adjoint_free(AdjointWork &w) {
    hipFree(w.lamface);
    hipFree(w.fwdface);
    hipFree(w.lamout);
    w = AdjointWork();
}

}  // namespace aderdg
