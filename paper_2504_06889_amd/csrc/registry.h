// Registry of the compiled kernel instances, keyed by (PDE, dim, order).
#pragma once
#include "kernels.h"

namespace aderdg {

using StepFn = void (*)(const StepArgs &, hipStream_t);
using MaxEigFn = void (*)(const void *, int, const PdeArgs &, long, unsigned long long *, hipStream_t);

struct KernelSet {
    StepFn pred[4] = {nullptr, nullptr, nullptr, nullptr};  // by predictor precision
    StepFn fused[4] = {nullptr, nullptr, nullptr, nullptr}; // corrector of the previous step + predictor
    StepFn corr[4] = {nullptr, nullptr, nullptr, nullptr};  // by face (flux) precision
    MaxEigFn maxeig = nullptr;
    int V = 0, cpb = 0, tpb = 0;
};

void register_kernels(int pde, int dim, int order, const KernelSet &ks);
const KernelSet *find_kernels(int pde, int dim, int order);

template <class Pde, int DIM, int N>
struct Instance {
    using Sh = Shape<DIM, N>;
    static long grid(long ncell) { return (ncell + Sh::CPB - 1) / Sh::CPB; }
    template <int PP>
    static void pred(const StepArgs &a, hipStream_t st) {
        hipLaunchKernelGGL((k_predictor<Pde, DIM, N, PP, false>), dim3(grid(a.ncell)), dim3(Sh::TPB), 0, st, a);
    }
    template <int PP>
    static void fused(const StepArgs &a, hipStream_t st) {
        hipLaunchKernelGGL((k_predictor<Pde, DIM, N, PP, true>), dim3(grid(a.ncell)), dim3(Sh::TPB), 0, st, a);
    }
    template <int FP>
    static void corr(const StepArgs &a, hipStream_t st) {
        hipLaunchKernelGGL((k_corrector<Pde, DIM, N, FP>), dim3(grid(a.ncell)), dim3(Sh::TPB), 0, st, a);
    }
    static void maxeig(const void *Q, int sp, const PdeArgs &p, long ncell, unsigned long long *out,
                       hipStream_t st) {
        long total = ncell * Sh::S;
        long g = (total + 255) / 256;
        if (g > 4096) g = 4096;
        hipLaunchKernelGGL((k_maxeig<Pde, DIM, N>), dim3(g), dim3(256), 0, st, Q, sp, p, ncell, out);
    }
    Instance(int pde, bool mixed) {
        KernelSet ks;
        ks.pred[P64] = &pred<P64>;
        ks.fused[P64] = &fused<P64>;
        if (mixed) {
            ks.pred[P32] = &pred<P32>;
            ks.pred[PBF16] = &pred<PBF16>;
            ks.pred[PF16] = &pred<PF16>;
            ks.fused[P32] = &fused<P32>;
            ks.fused[PBF16] = &fused<PBF16>;
            ks.fused[PF16] = &fused<PF16>;
        }
        ks.corr[P64] = &corr<P64>;
        ks.corr[P32] = &corr<P32>;
        ks.corr[PBF16] = &corr<PBF16>;
        ks.corr[PF16] = &corr<PF16>;
        ks.maxeig = &maxeig;
        ks.V = Pde::V;
        ks.cpb = Sh::CPB;
        ks.tpb = Sh::TPB;
        register_kernels(pde, DIM, N, ks);
    }
};

}  // namespace aderdg
