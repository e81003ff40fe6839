// Discrete adjoint of the ADER-DG step for acoustics with per-cell material.
#pragma once
#include <string>

#include "common.h"
#include "kernels.h"

namespace aderdg {

struct AdjointArgs {
    void (*pred)(const StepArgs &, hipStream_t);  // forward predictor of this shape in the predictor format
    int cfg_pde, dim, order;
    long ncell;
    int cells[3];
    const DevBasis *B;
    const ScaledTime *st;  // the time operator scaled by -sigma for dt (forward predictor)
    PdeArgs pde;
    double dt, t, inv_h, sigma;
    int iters;
    const double *Qn;
    const void *fwdface;  // forward face data of the step, or null: recomputed from Qn
    double *lam;
    double *grad;
    long src_cell;
    const double *src_phi;
    double src_f0, src_t0, src_amp;
    double src_s[kMaxN], src_bar;  // the forward predictor's source values (StepArgs)
    int prec_pred, prec_vol;       // contraction formats (Prec): both P64, or both lower
};

// Device work buffers owned by a solver for the adjoint.
struct AdjointWork {
    void *lamface = nullptr;   // face restrictions of the incoming adjoint
    void *fwdface = nullptr;   // forward face data of the step
    double *lamout = nullptr;  // outgoing adjoint
    size_t bytes_lamface = 0, bytes_fwdface = 0, bytes_lamout = 0;
};

// One adjoint step.  lamface_scratch: device memory of at least
// adjoint_lamface_bytes(a) bytes for the face restrictions of the incoming
// adjoint (then nothing is allocated; a.fwdface must be given), or null: the
// solver's work buffers, allocated on first use.
int adjoint_step(AdjointWork &w, const AdjointArgs &a, hipStream_t st, std::string &msg,
                 void *lamface_scratch = nullptr);
size_t adjoint_lamface_bytes(const AdjointArgs &a);

// The library's static scratch array for callers that cannot allocate:
// noalloc_scratch_init() resolves its address on the current device (once per
// device; call with that device current), noalloc_scratch() returns it
// (null if not resolved).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
int noalloc_scratch_init(std::string &msg);
void *noalloc_scratch(int device);
void adjoint_free(AdjointWork &w);
// Receiver misfit scatter, grouped by cell: ncells cells ucell[m] hold the
// receivers order[start[m] .. start[m+1]-1].
void receivers_adjoint(double *lam, int V, int S, int n, int dim, int ncells, const long *ucell, const int *start,
                       const int *order, const double *rphi, const double *weight, hipStream_t st);

}  // namespace aderdg
