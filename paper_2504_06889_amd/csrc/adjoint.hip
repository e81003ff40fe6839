// Discrete adjoint of the ADER-DG step (acoustics, per-cell sound speed).
#include "adjoint.h"

#include "aderdg.h"

namespace aderdg {

// lam[cell_r][0][s] += weight[r] * prod_j phi[r][j][i_j(s)]  (one thread per receiver and node)
__global__ void k_receivers_adjoint(double *lam, int V, int S, int n, int dim, int nrec, const long *rcell,
                                    const double *rphi, const double *weight) {
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= (long)nrec * S) return;
    const int r = i / S, s = i % S;
    const double *ph = rphi + (long)r * 3 * kMaxN;
    double w = ph[s % n];
    if (dim > 1) w *= ph[kMaxN + (s / n) % n];
    if (dim > 2) w *= ph[2 * kMaxN + s / (n * n)];
    atomicAdd(lam + rcell[r] * V * S + s, weight[r] * w);
}

void receivers_adjoint(double *lam, int V, int S, int n, int dim, int nrec, const long *rcell, const double *rphi,
                       const double *weight, hipStream_t st) {
    const long total = (long)nrec * S;
    hipLaunchKernelGGL(k_receivers_adjoint, dim3((total + 255) / 256), dim3(256), 0, st, lam, V, S, n, dim, nrec,
                       rcell, rphi, weight);
}

int adjoint_step(AdjointWork &, const AdjointArgs &, hipStream_t, std::string &msg) {
    msg = "adjoint step not built";
    return ADERDG_E_UNSUPPORTED;
}

void adjoint_free(AdjointWork &w) {
    hipFree(w.lamface);
    hipFree(w.fwdface);
    hipFree(w.lamout);
    w = AdjointWork();
}

}  // namespace aderdg
