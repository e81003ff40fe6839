// HIP kernels of the ADER-DG time step (arXiv 2504.06889, Alg. 1) for gfx950.
//
//  k_predictor: one workgroup per CPB cells, one thread per spatial node.
//    Each thread keeps its node's space-time column q[a][v] (all time nodes,
//    all variables) in registers.  Per Picard iteration and time slice b the
//    pointwise fluxes F_j(q_b) are written to LDS, every 1-D line is
//    differentiated (D along x, y, z: in place in FP64 on the vector ALU, or
//    on the matrix cores in FP32/BF16/FP16 with FP32 accumulation), and the
//    owner thread folds the divergence into the FP64 Picard update
//    q_a <- Q - dt sum_b Atau[a][b] R_b (eq. Picard at the nodes).  The
//    epilogue forms the FP64 time averages, projects q and F_j to the 2d faces
//    (Alg. 1 "expansion") and adds the volume integral to Q.
//  k_corrector: per cell, the Rusanov flux on each face node of its 2d faces
//    (eq. rusanov_flux; well-balanced form for shallow water) and the face
//    integral (lift) into Q in FP64.
//  Face buffer: faces[cell][dir][side][q|f][var][face node] in the FLUX format.
#pragma once

#include <type_traits>

#include "common.h"

namespace aderdg {

struct StepArgs {
    double *Q;            // state [ncell][V][S]
    void *faces;          // face buffer
    const DevBasis *B;
    PdeArgs pde;
    long ncell;
    int cells[3];
    double dt, inv_h, sigma, t, h;
    int vol_prec, flux_prec;
    int iters;            // Picard iterations
    int write_state;      // 0: only the face data is produced (Q untouched)
    long src_cell;        // -1: no source
    const double *src_phi;
    double src_f0, src_t0, src_amp;
};

// Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// range of cells so that neighbouring cells share an L2.
__device__ __forceinline__ long xcd_block(long b, long G) {
    const long q = G / 8, r = G % 8, k = b % 8;
    return k * q + (k < r ? k : r) + b / 8;
}

__device__ __forceinline__ double ricker(double t, double f0, double t0, double amp) {
    const double pi = 3.14159265358979323846;
    const double x = pi * f0 * (t - t0);
    const double a = x * x;
    return amp * (1.0 - 2.0 * a) * exp(-a);
}

__device__ __forceinline__ long neighbour(long cell, int j, int dir, const int *cells, int dim) {
    long c0 = cell % cells[0];
    long rest = cell / cells[0];
    long c1 = dim > 1 ? rest % cells[1] : 0;
    long c2 = dim > 2 ? rest / cells[1] : 0;
    if (j == 0) c0 = (c0 + dir + cells[0]) % cells[0];
    if (j == 1) c1 = (c1 + dir + cells[1]) % cells[1];
    if (j == 2) c2 = (c2 + dir + cells[2]) % cells[2];
    return c0 + (long)cells[0] * (c1 + (long)cells[1] * c2);
}

// ---------------------------------------------------------------------------
// FP64 line pass: X <- M along each line, in place (vector ALU).
// Lines are enumerated as (blk, f): blk indexes a block of S values, f the
// face node through which the line runs; the direction of block blk is
// dir_of(blk).
// ---------------------------------------------------------------------------
template <int n, int S, int F, class DirOf>
__device__ __forceinline__ void lines_fp64(double *X, int nblk, const double (*M)[kMaxN], DirOf dir_of,
                                           int tid, int nthreads) {
    const int NL = nblk * F;
    for (int L = tid; L < NL; L += nthreads) {
        const int f = L % F, blk = L / F;
        const int j = dir_of(blk);
        const int st = j == 0 ? 1 : (j == 1 ? n : n * n);
        double *base = X + (long)blk * S + line_start<n>(f, j);
        double x[n];
#pragma unroll
        for (int k = 0; k < n; k++) x[k] = base[k * st];
#pragma unroll
        for (int i = 0; i < n; i++) {
            double y = 0.0;
#pragma unroll
            for (int k = 0; k < n; k++) y = fma(M[i][k], x[k], y);
            base[i * st] = y;
        }
    }
}

// ---------------------------------------------------------------------------
// Matrix-core line pass: Y = M along each line, inputs in format P (FP32,
// BF16 or FP16), FP32 accumulation.  Each 16x16 MFMA tile holds LPR lines per
// row: the row's K entries are LPR line segments of NB values, and the B
// operand is the block-diagonal matrix diag(M^T, ..., M^T) (LPR blocks of
// NB x NB, zero padded beyond n).  One tile thus differentiates 16*LPR lines.
// Lane layouts (16x16xK, 64 lanes): A[row = lane%16][k = kw*(lane/16) + e],
// B[k = kw*(lane/16) + e][col = lane%16], C[row = 4*(lane/16) + e][col = lane%16].
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

template <int P, int n, int S, int F, class DirOf>
__device__ __forceinline__ void lines_mfma(const typename Store<P>::T *X, float *Y, int nblk,
                                           const float (*M)[kMaxN], DirOf dir_of, int tid,
                                           int nthreads) {
    using T = typename Store<P>::T;
    constexpr int NB = n <= 4 ? 4 : 8;   // line segment length in the tile
    constexpr int LPR = 16 / NB;         // lines per tile row
    constexpr int LPT = 16 * LPR;        // lines per tile
    const int NL = nblk * F;
    const int ntiles = (NL + LPT - 1) / LPT;
    const int lane = tid & 63, wave = tid >> 6, nwave = nthreads >> 6;
    const int r = lane & 15, g = lane >> 4;

    // B operand (constant): B[k][col] = M[col%NB][k%NB] on diagonal blocks
    auto bval = [&](int k) -> float {
        const int kb = k / NB, kk = k % NB, cb = r / NB, cc = r % NB;
        return (kb == cb && kk < n && cc < n) ? M[cc][kk] : 0.0f;
    };
    // address of position p of line L (or -1)
    auto addr = [&](int L, int p) -> int {
        if (L >= NL || p >= n) return -1;
        const int f = L % F, blk = L / F;
        const int j = dir_of(blk);
        const int st = j == 0 ? 1 : (j == 1 ? n : n * n);
        return blk * S + line_start<n>(f, j) + p * st;
    };

    if constexpr (P == P32) {
        float b[4];
#pragma unroll
        for (int m = 0; m < 4; m++) b[m] = bval(4 * m + g);
        for (int tile = wave; tile < ntiles; tile += nwave) {
            const int L0 = tile * LPT;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int m = 0; m < 4; m++) {
                const int k = 4 * m + g;
                const int ad = addr(L0 + LPR * r + k / NB, k % NB);
                const float av = ad >= 0 ? X[ad] : 0.0f;
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b[m], acc, 0, 0, 0);
            }
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int ad = addr(L0 + LPR * (4 * g + e) + r / NB, r % NB);
                if (ad >= 0) Y[ad] = acc[e];
            }
        }
    } else {
        // 16x16x16 (bf16 / fp16): lane holds k = 4g .. 4g+3
        T bb[4];
#pragma unroll
        for (int e = 0; e < 4; e++) bb[e] = round_to<P>(bval(4 * g + e));
        for (int tile = wave; tile < ntiles; tile += nwave) {
            const int L0 = tile * LPT;
            T aa[4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int k = 4 * g + e;
                const int ad = addr(L0 + LPR * r + k / NB, k % NB);
                aa[e] = ad >= 0 ? X[ad] : round_to<P>(0.0f);
            }
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            if constexpr (P == PBF16) {
                i16x4 av, bv;
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    av[e] = __builtin_bit_cast(short, aa[e]);
                    bv[e] = __builtin_bit_cast(short, bb[e]);
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
            } else {
                f16x4 av, bv;
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    av[e] = aa[e];
                    bv[e] = bb[e];
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16f16(av, bv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int ad = addr(L0 + LPR * (4 * g + e) + r / NB, r % NB);
                if (ad >= 0) Y[ad] = acc[e];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Picard line buffers.  Lines are numbered ((cb*DIM + j)*NV + v)*F + f: block
// cell cb, direction j, variable v (NV = V, plus eta for the non-conservative
// term), face node f.
//  FP64:  position-major X[k][line] with an odd pitch NLP (conflict-free
//         column access by consecutive lines), separate input and output.
//  other: line-major F[line][NB] (NB = 4 or 8 positions, zero padded) in the
//         contraction format, so that a lane's 4 MFMA operand values are one
//         8-byte load; FP32 results in the same layout.
// ---------------------------------------------------------------------------
template <class Pde, int DIM, int N, int PP>
struct PicardLayout {
    using Sh = Shape<DIM, N>;
    static constexpr int n = Sh::n, F = Sh::F, CPB = Sh::CPB;
    static constexpr int NV = Pde::kNCP ? Pde::V + 1 : Pde::V;
    static constexpr int NL = CPB * DIM * NV * F;
    static constexpr int NLP = NL | 1;
    static constexpr int NB = n <= 4 ? 4 : 8;
    static constexpr int LPR = 16 / NB;
    static constexpr int LPT = 16 * LPR;
    static constexpr int NTILE = (NL + LPT - 1) / LPT;
    static constexpr int NLT = NTILE * LPT;
    // element offset of position k on line `line`, and the offset between variables
    __device__ static constexpr int elem(int line, int k) { return PP == P64 ? k * NLP + line : line * NB + k; }
    static constexpr int VSTRIDE = PP == P64 ? F : F * NB;
    // FP32 output layout of the matrix-core path: line-major with a padded line
    // stride OSTRIDE = NB + NB/4, so that the four lane groups of a tile (whose
    // rows are 4*LPR lines apart) write to different LDS banks.
    static constexpr int OSTRIDE = NB + NB / 4;
    static constexpr int OVSTRIDE = F * OSTRIDE;
    static constexpr int OTILE = LPT * OSTRIDE;
    __device__ static constexpr int oelem(int line, int k) { return line * OSTRIDE + k; }
    static constexpr size_t obytes = (size_t)NTILE * OTILE * 4;
    static constexpr size_t bytes =
        PP == P64 ? (size_t)2 * n * NLP * 8 : (size_t)NLT * NB * sizeof(typename Store<PP>::T) + obytes;
};

// ---------------------------------------------------------------------------
// LDS budget of the predictor
// ---------------------------------------------------------------------------
template <class Pde, int DIM, int N, int PP>
struct PredLds {
    using Sh = Shape<DIM, N>;
    static constexpr int V = Pde::V;
    static constexpr int NV = Pde::kNCP ? V + 1 : V;
    static constexpr int CPB = Sh::CPB, S = Sh::S;
    static constexpr size_t picard = PicardLayout<Pde, DIM, N, PP>::bytes;
    // epilogue: qbar, fbar_j (double), volume staging (4-byte input + float output)
    static constexpr size_t epi = (size_t)CPB * V * S * (8 + 8 + 4 + 4);
    static constexpr size_t ncp = Pde::kNCP ? (size_t)CPB * DIM * S * 8 : 0;
    static constexpr size_t bytes0 = picard > epi ? picard : epi;
    static constexpr size_t bytes = bytes0 > ncp ? bytes0 : ncp;
};

// Target occupancy of the predictor: the lower-precision paths keep the
// Picard iterate in FP32 registers and can run two wavefronts per SIMD when
// their LDS allows two workgroups per CU.
template <class Pde, int DIM, int N, int PP>
struct PredOcc {
    static constexpr int waves =
        (PP != P64 && PredLds<Pde, DIM, N, PP>::bytes * 2 <= 160 * 1024 && Shape<DIM, N>::TPB <= 256) ? 2 : 1;
};

// Volume contribution along direction j in a lower format PV: round fbar_j,
// matrix-core line pass with Kxi, accumulate into vol (FP64).
template <class Pde, int DIM, int N, int PV>
__device__ __forceinline__ void volume_dir_mixed(char *stage, const double *fbj_reg, double *vol,
                                                 int j, int cb, int s, bool slot, bool active,
                                                 const DevBasis *B, int tid) {
    using Sh = Shape<DIM, N>;
    constexpr int n = Sh::n, S = Sh::S, F = Sh::F, CPB = Sh::CPB, TPB = Sh::TPB, V = Pde::V;
    using T = typename Store<PV>::T;
    T *in = reinterpret_cast<T *>(stage);
    float *out = reinterpret_cast<float *>(stage + (size_t)CPB * V * S * 4);
    if (slot) {
#pragma unroll
        for (int v = 0; v < V; v++) in[(cb * V + v) * S + s] = round_to<PV>(active ? (float)fbj_reg[v] : 0.0f);
    }
    __syncthreads();
    lines_mfma<PV, n, S, F>(in, out, CPB * V, B->Kxip[PV], [j](int) { return j; }, tid, TPB);
    __syncthreads();
    if (active) {
#pragma unroll
        for (int v = 0; v < V; v++) vol[v] += (double)out[(cb * V + v) * S + s];
    }
}

// Store one projected face value in the FLUX format.
template <int FP>
__device__ __forceinline__ void face_store(void *faces, long idx, double val) {
    using T = typename FaceT<FP>::T;
    reinterpret_cast<T *>(faces)[idx] = round_to<FP>((float)val);
}
template <>
__device__ __forceinline__ void face_store<P64>(void *faces, long idx, double val) {
    reinterpret_cast<double *>(faces)[idx] = val;
}

// Projection of one line onto a face (Alg. 1 "expansion"): FP64 or inputs
// rounded to FP and FP32 accumulation.
template <int FP, int n>
__device__ __forceinline__ double face_project(const double *src, int st, const DevBasis *B, int side) {
    if constexpr (FP == P64) {
        const double *E = side ? B->F1 : B->F0;
        double y = 0.0;
#pragma unroll
        for (int k = 0; k < n; k++) y = fma(E[k], src[k * st], y);
        return y;
    } else {
        const float *E = side ? B->F1p[FP] : B->F0p[FP];
        float y = 0.0f;
#pragma unroll
        for (int k = 0; k < n; k++) y += E[k] * widen(round_to<FP>((float)src[k * st]));
        return (double)y;
    }
}

// ---------------------------------------------------------------------------
// Predictor + face projection + volume integral (Alg. 1, first traversal)
// ---------------------------------------------------------------------------
template <class Pde, int DIM, int N, int PP>
__global__ __launch_bounds__((Shape<DIM, N>::TPB))
__attribute__((amdgpu_waves_per_eu(PredOcc<Pde, DIM, N, PP>::waves, 8))) void k_predictor(StepArgs a) {
    using Sh = Shape<DIM, N>;
    using L = PredLds<Pde, DIM, N, PP>;
    constexpr int n = Sh::n, S = Sh::S, F = Sh::F, CPB = Sh::CPB, TPB = Sh::TPB;
    constexpr int V = Pde::V, NV = L::NV;
    __shared__ __attribute__((aligned(16))) char smem[L::bytes];

    const DevBasis *B = a.B;
    const int tid = threadIdx.x;
    const int cb = tid / S, s = tid % S;
    const long blk = xcd_block(blockIdx.x, gridDim.x);
    const long cell0 = blk * CPB;
    const long cell = cell0 + cb;
    const bool slot = cb < CPB;               // thread owns an LDS node slot
    const bool active = slot && cell < a.ncell;  // ... of a real cell
    const typename Pde::Coef coef = Pde::cell(a.pde, active ? cell : 0);

    double Qn[V];
#pragma unroll
    for (int v = 0; v < V; v++) Qn[v] = active ? a.Q[(cell * V + v) * S + s] : 1.0;
    // The final Picard iterate is q_a = Qn - (dt/h) acc[a] (acc of the last
    // iteration accumulates Atau applied to h R_b); the epilogue evaluates it
    // on the fly from acc.

    const bool src_here = active && cell == a.src_cell;
    const double src_phi = src_here ? a.src_phi[s] : 0.0;
    const int iters = a.iters;

    // ---------------- Picard iterations (eq. Picard) ----------------
    // Per slice b: the node owners write F_j(q_b) into the line buffer, every
    // line is differentiated, and the owners gather sum_j D_j F_j at their
    // node and fold it into acc[a] += Atau[a][b] R_b.  Two barriers per slice:
    // the line pass reads a buffer the owners do not touch until the next
    // slice's first barrier, and writes one they only read after the second.
    using PL = PicardLayout<Pde, DIM, N, PP>;
    double acc[n][V];
    // per-thread offset of its node in each direction's lines (variable 0)
    int po[DIM], pr[DIM];
#pragma unroll
    for (int j = 0; j < DIM; j++) {
        const int line0 = ((cb * DIM + j) * NV) * F + face_of<n, DIM>(s, j);
        po[j] = PL::elem(line0, coord<n>(s, j));
        pr[j] = PL::oelem(line0, coord<n>(s, j));
    }
    if constexpr (PP == P64) {
        double *Xin = reinterpret_cast<double *>(smem);   // [n][NLP] position-major
        double *Xout = Xin + n * PL::NLP;
        double q[n][V];
#pragma unroll
        for (int t = 0; t < n; t++)
#pragma unroll
            for (int v = 0; v < V; v++) q[t][v] = Qn[v];
#pragma unroll 1
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int t = 0; t < n; t++)
#pragma unroll
                for (int v = 0; v < V; v++) acc[t][v] = 0.0;
#pragma unroll
            for (int b = 0; b < n; b++) {
                // Padding cells (beyond ncell) hold Qn = 1 and never update it, so
                // their fluxes are finite: no stale or non-finite bits enter the lines.
                if (slot) {
#pragma unroll
                    for (int j = 0; j < DIM; j++) {
                        double Fv[V];
                        Pde::flux(coef, q[b], j, Fv);
#pragma unroll
                        for (int v = 0; v < V; v++) Xin[po[j] + v * PL::VSTRIDE] = Fv[v];
                        if constexpr (Pde::kNCP) Xin[po[j] + V * PL::VSTRIDE] = Pde::ncp_input(q[b]);
                    }
                }
                __syncthreads();
                for (int Ln = tid; Ln < PL::NL; Ln += TPB) {
                    double x[n];
#pragma unroll
                    for (int k = 0; k < n; k++) x[k] = Xin[k * PL::NLP + Ln];
#pragma unroll
                    for (int i = 0; i < n; i++) {
                        double y = 0.0;
#pragma unroll
                        for (int k = 0; k < n; k++) y = fma(B->D[i][k], x[k], y);
                        Xout[i * PL::NLP + Ln] = y;
                    }
                }
                __syncthreads();
                if (active) {
                    // h R_b: the 1/h of R_b is folded into sigma = dt/h of the update
#pragma unroll
                    for (int v = 0; v < V; v++) {
                        double r = 0.0;
#pragma unroll
                        for (int j = 0; j < DIM; j++) r += Xout[po[j] + v * PL::VSTRIDE];
                        if constexpr (Pde::kNCP) {
                            if (v >= 1 && v <= DIM) r += coef.g * q[b][0] * Xout[po[v - 1] + V * PL::VSTRIDE];
                        }
                        if (v == 0 && src_here) r -= a.h * ricker(a.t + B->xi[b] * a.dt, a.src_f0, a.src_t0, a.src_amp) * src_phi;
#pragma unroll
                        for (int t = 0; t < n; t++) acc[t][v] = fma(B->Atau[t][b], r, acc[t][v]);
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < n; t++)
#pragma unroll
                for (int v = 0; v < V; v++) q[t][v] = fma(-a.sigma, acc[t][v], Qn[v]);
        }
    } else {
        using T = typename Store<PP>::T;
        constexpr int NB = PL::NB, LPR = PL::LPR, LPT = PL::LPT;
        T *Fb = reinterpret_cast<T *>(smem);                                    // [NLT][NB] line-major
        float *Rb = reinterpret_cast<float *>(smem + (size_t)PL::NLT * NB * sizeof(T));  // skewed [NLT][NB]
        // zero padding (positions >= n and lines >= NL are never written)
        for (int i = tid; i < PL::NLT * NB; i += TPB) Fb[i] = round_to<PP>(0.0f);
        const int lane = tid & 63, wave = tid >> 6;
        constexpr int NWAVE = TPB / 64;
        const int r = lane & 15, g = lane >> 4;
        // lane-constant operand offsets inside a tile (elements)
        // output offset in the skewed FP32 layout (lane groups g land on different banks)
        const int coff_o = PL::oelem(LPR * 4 * g + r / NB, r % NB);
        // B operand: block-diagonal D^T, B[k][col] = D[col % NB][k % NB] on diagonal blocks
        auto bval = [&](int k) -> float {
            const int kb = k / NB, kk = k % NB, cbk = r / NB, cc = r % NB;
            return (kb == cbk && kk < n && cc < n) ? B->Dp[PP][cc][kk] : 0.0f;
        };
        // constant B operands and lane offsets, set up once
        float bm[4];      // FP32 path: B[4m+g][r]
        int aoffm[4];     // FP32 path: A offsets of the four K=4 steps
#pragma unroll
        for (int m = 0; m < 4; m++) {
            const int k = 4 * m + g;
            bm[m] = bval(k);
            aoffm[m] = (LPR * r + k / NB) * NB + k % NB;
        }
        const int aoff = (LPR * r + (4 * g) / NB) * NB + (4 * g) % NB;  // 16-bit paths
        typename std::conditional<PP == PBF16, i16x4, f16x4>::type bvec;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const T be = round_to<PP>(bval(4 * g + e));
            if constexpr (PP == PBF16) bvec[e] = __builtin_bit_cast(short, be);
            else if constexpr (PP == PF16) bvec[e] = be;
        }
        float qf[n][V];
#pragma unroll
        for (int t = 0; t < n; t++)
#pragma unroll
            for (int v = 0; v < V; v++) qf[t][v] = (float)Qn[v];
#pragma unroll 1
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int t = 0; t < n; t++)
#pragma unroll
                for (int v = 0; v < V; v++) acc[t][v] = 0.0;
#pragma unroll
            for (int b = 0; b < n; b++) {
                const float *qb = qf[b];
                // padding cells: finite fluxes of Qn = 1 (see the FP64 branch)
                if (slot) {
#pragma unroll
                    for (int j = 0; j < DIM; j++) {
                        float Fv[V];
                        Pde::flux(coef, qb, j, Fv);
#pragma unroll
                        for (int v = 0; v < V; v++) Fb[po[j] + v * PL::VSTRIDE] = round_to<PP>(Fv[v]);
                        if constexpr (Pde::kNCP) Fb[po[j] + V * PL::VSTRIDE] = round_to<PP>(Pde::ncp_input(qb));
                    }
                }
                __syncthreads();
                if constexpr (PP == P32) {
                    for (int tile = wave; tile < PL::NTILE; tile += NWAVE) {
                        const int base = tile * LPT * NB;
                        const int obase = tile * PL::OTILE;
                        f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int m = 0; m < 4; m++)
                            c = __builtin_amdgcn_mfma_f32_16x16x4f32(Fb[base + aoffm[m]], bm[m], c, 0, 0, 0);
#pragma unroll
                        for (int e = 0; e < 4; e++) Rb[obase + coff_o + LPR * PL::OSTRIDE * e] = c[e];
                    }
                } else {
                    // tiles of this wave in batches of TB: all operand loads, then the
                    // independent MFMAs, then the stores, so that LDS and matrix-core
                    // latencies overlap
                    constexpr int TPW = (PL::NTILE + NWAVE - 1) / NWAVE;
                    constexpr int TB = TPW < 4 ? TPW : 4;
#pragma unroll
                    for (int k0 = 0; k0 < TPW; k0 += TB) {
                        using VT = typename std::conditional<PP == PBF16, i16x4, f16x4>::type;
                        VT av[TB];
                        f32x4 cc[TB];
#pragma unroll
                        for (int k = 0; k < TB; k++) {
                            const int tile = wave + (k0 + k) * NWAVE;
                            if (k0 + k < TPW && tile < PL::NTILE)
                                av[k] = *reinterpret_cast<const VT *>(Fb + tile * LPT * NB + aoff);
                        }
#pragma unroll
                        for (int k = 0; k < TB; k++) {
                            const int tile = wave + (k0 + k) * NWAVE;
                            if (k0 + k < TPW && tile < PL::NTILE) {
                                f32x4 z = {0.f, 0.f, 0.f, 0.f};
                                if constexpr (PP == PBF16)
                                    cc[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[k], bvec, z, 0, 0, 0);
                                else
                                    cc[k] = __builtin_amdgcn_mfma_f32_16x16x16f16(av[k], bvec, z, 0, 0, 0);
                            }
                        }
#pragma unroll
                        for (int k = 0; k < TB; k++) {
                            const int tile = wave + (k0 + k) * NWAVE;
                            if (k0 + k < TPW && tile < PL::NTILE) {  // padding lanes store to unused slots
                                const int obase = tile * PL::OTILE;
#pragma unroll
                                for (int e = 0; e < 4; e++) Rb[obase + coff_o + LPR * PL::OSTRIDE * e] = cc[k][e];
                            }
                        }
                    }
                }
                __syncthreads();
                if (active) {
                    // R_b[v] = (1/h) sum_j (D_j F_j)[v] (- source), folded straight into
                    // acc[a][v] += Atau[a][b] R_b[v] one variable at a time
#pragma unroll
                    for (int v = 0; v < V; v++) {
                        // the divergence sum over directions is part of the FP32
                        // contraction; h R_b is accumulated (1/h folded into sigma)
                        float rf = 0.0f;
#pragma unroll
                        for (int j = 0; j < DIM; j++) rf += Rb[pr[j] + v * PL::OVSTRIDE];
                        double rr = (double)rf;
                        if constexpr (Pde::kNCP) {
                            if (v >= 1 && v <= DIM)
                                rr += (double)((float)coef.g * qb[0] * Rb[pr[v - 1] + V * PL::OVSTRIDE]);
                        }
                        if (v == 0 && src_here)
                            rr -= a.h * ricker(a.t + B->xi[b] * a.dt, a.src_f0, a.src_t0, a.src_amp) * src_phi;
#pragma unroll
                        for (int t = 0; t < n; t++) acc[t][v] = fma(B->Atau[t][b], rr, acc[t][v]);
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < n; t++)
#pragma unroll
                for (int v = 0; v < V; v++) qf[t][v] = (float)fma(-a.sigma, acc[t][v], Qn[v]);
        }
    }
    __syncthreads();

    // ---------------- time averages (FP64) ----------------
    // qbar here; the flux averages fbar_j are formed per direction below
    double qbar[V], nbar[V];
#pragma unroll
    for (int v = 0; v < V; v++) {
        qbar[v] = 0.0;
        nbar[v] = 0.0;
#pragma unroll
        for (int t = 0; t < n; t++) qbar[v] = fma(B->w[t], fma(-a.sigma, acc[t][v], Qn[v]), qbar[v]);
    }
    if constexpr (Pde::kNCP) {
        // average of the non-conservative product: sum_a w_a g h_a D_j eta_a
        double *eb = reinterpret_cast<double *>(smem);  // [CPB][DIM][S]
#pragma unroll
        for (int t = 0; t < n; t++) {
            double qt[V];
#pragma unroll
            for (int v = 0; v < V; v++) qt[v] = fma(-a.sigma, acc[t][v], Qn[v]);
            if (slot) {
#pragma unroll
                for (int j = 0; j < DIM; j++) eb[(cb * DIM + j) * S + s] = active ? Pde::ncp_input(qt) : 0.0;
            }
            __syncthreads();
            lines_fp64<n, S, F>(eb, CPB * DIM, B->D, [](int blk_) { return blk_ % DIM; }, tid, TPB);
            __syncthreads();
            if (active) {
#pragma unroll
                for (int j = 0; j < DIM; j++)
                    nbar[1 + j] = fma(B->w[t], coef.g * qt[0] * eb[(cb * DIM + j) * S + s], nbar[1 + j]);
            }
            __syncthreads();
        }
    }

    // ---------------- face projection and volume integral ----------------
    double *QB = reinterpret_cast<double *>(smem);              // [CPB][V][S]
    double *FB = QB + (size_t)CPB * V * S;                      // [CPB][V][S]
    char *stage = reinterpret_cast<char *>(FB + (size_t)CPB * V * S);
    if (slot) {
#pragma unroll
        for (int v = 0; v < V; v++) QB[(cb * V + v) * S + s] = active ? qbar[v] : 0.0;
    }
    double vol[V];
#pragma unroll
    for (int v = 0; v < V; v++) vol[v] = 0.0;

#pragma unroll 1
    for (int j = 0; j < DIM; j++) {
        // fbar_j = sum_a w_a F_j(q_a) from the final iterate q_a = Qn - dt acc[a]
        double fbj[V];
#pragma unroll
        for (int v = 0; v < V; v++) fbj[v] = 0.0;
#pragma unroll
        for (int t = 0; t < n; t++) {
            double qt[V], Fv[V];
#pragma unroll
            for (int v = 0; v < V; v++) qt[v] = fma(-a.sigma, acc[t][v], Qn[v]);
            Pde::flux(coef, qt, j, Fv);
#pragma unroll
            for (int v = 0; v < V; v++) fbj[v] = fma(B->w[t], Fv[v], fbj[v]);
        }
        if (slot) {
#pragma unroll
            for (int v = 0; v < V; v++) FB[(cb * V + v) * S + s] = active ? fbj[v] : 0.0;
        }
        __syncthreads();
        // faces of direction j: items (cb, side, q|f, v, f)
        {
            const int st = j == 0 ? 1 : (j == 1 ? n : n * n);
            constexpr int NFI = CPB * 2 * 2 * V * F;
            for (int itm = tid; itm < NFI; itm += TPB) {
                const int f = itm % F;
                int rr = itm / F;
                const int v = rr % V;
                rr /= V;
                const int qf = rr % 2;
                rr /= 2;
                const int side = rr % 2;
                const int cbi = rr / 2;
                const long c = cell0 + cbi;
                if (c >= a.ncell) continue;
                const double *src = (qf == 0 ? QB : FB) + (cbi * V + v) * S + line_start<n>(f, j);
                const long idx = ((((c * DIM + j) * 2 + side) * 2 + qf) * V + v) * (long)F + f;
                switch (a.flux_prec) {
                case P64: face_store<P64>(a.faces, idx, face_project<P64, n>(src, st, B, side)); break;
                case P32: face_store<P32>(a.faces, idx, face_project<P32, n>(src, st, B, side)); break;
                case PBF16: face_store<PBF16>(a.faces, idx, face_project<PBF16, n>(src, st, B, side)); break;
                default: face_store<PF16>(a.faces, idx, face_project<PF16, n>(src, st, B, side)); break;
                }
            }
        }
        // volume along j
        if (a.vol_prec == P64) {
            if (active) {
                const int i = coord<n>(s, j);
                const int st = j == 0 ? 1 : (j == 1 ? n : n * n);
#pragma unroll
                for (int v = 0; v < V; v++) {
                    const double *line = FB + (cb * V + v) * S + (s - i * st);
                    double y = 0.0;
#pragma unroll
                    for (int k = 0; k < n; k++) y = fma(B->Kxi[i][k], line[k * st], y);
                    vol[v] += y;
                }
            }
        } else if (a.vol_prec == P32) {
            volume_dir_mixed<Pde, DIM, N, P32>(stage, fbj, vol, j, cb, s, slot, active, B, tid);
        } else if (a.vol_prec == PBF16) {
            volume_dir_mixed<Pde, DIM, N, PBF16>(stage, fbj, vol, j, cb, s, slot, active, B, tid);
        } else {
            volume_dir_mixed<Pde, DIM, N, PF16>(stage, fbj, vol, j, cb, s, slot, active, B, tid);
        }
        __syncthreads();
    }

    if (active && a.write_state) {
        double sbar = 0.0;
        if (src_here) {
#pragma unroll
            for (int t = 0; t < n; t++)
                sbar += B->w[t] * ricker(a.t + B->xi[t] * a.dt, a.src_f0, a.src_t0, a.src_amp);
        }
#pragma unroll
        for (int v = 0; v < V; v++) {
            double qn = Qn[v] + a.sigma * vol[v];
            if constexpr (Pde::kNCP) qn -= a.sigma * nbar[v];
            if (v == 0 && src_here) qn += a.dt * sbar * src_phi;
            a.Q[(cell * V + v) * S + s] = qn;
        }
    }
}

// ---------------------------------------------------------------------------
// Corrector: Riemann solve per face node and face integral (Alg. 1, second
// traversal).  FP is the face format; FP32 arithmetic when FP != FP64.
// ---------------------------------------------------------------------------
template <class Pde, int DIM, int N, int FP>
__global__ __launch_bounds__((Shape<DIM, N>::TPB)) void k_corrector(StepArgs a) {
    using Sh = Shape<DIM, N>;
    constexpr int n = Sh::n, S = Sh::S, F = Sh::F, CPB = Sh::CPB, TPB = Sh::TPB, V = Pde::V;
    using CT = typename std::conditional<FP == P64, double, float>::type;
    using FT = typename FaceT<FP>::T;
    __shared__ CT G[CPB * DIM * 2 * V * F];

    const DevBasis *B = a.B;
    const FT *faces = reinterpret_cast<const FT *>(a.faces);
    const int tid = threadIdx.x;
    const long blk = xcd_block(blockIdx.x, gridDim.x);
    const long cell0 = blk * CPB;

    constexpr int NRI = CPB * DIM * 2 * F;
    for (int itm = tid; itm < NRI; itm += TPB) {
        const int f = itm % F;
        int rr = itm / F;
        const int side = rr % 2;
        rr /= 2;
        const int j = rr % DIM;
        const int cbi = rr / DIM;
        const long c = cell0 + cbi;
        if (c >= a.ncell) continue;
        const long nb = neighbour(c, j, side ? 1 : -1, a.cells, DIM);
        const long cl = side ? c : nb, cr = side ? nb : c;
        CT qm[V], fm[V], qp[V], fp[V];
        const long bl = (((cl * DIM + j) * 2 + 1) * 2) * V * (long)F + f;
        const long br = (((cr * DIM + j) * 2 + 0) * 2) * V * (long)F + f;
#pragma unroll
        for (int v = 0; v < V; v++) {
            qm[v] = (CT)widen(faces[bl + (long)v * F]);
            fm[v] = (CT)widen(faces[bl + (long)(V + v) * F]);
            qp[v] = (CT)widen(faces[br + (long)v * F]);
            fp[v] = (CT)widen(faces[br + (long)(V + v) * F]);
        }
        const typename Pde::Coef kl = Pde::cell(a.pde, cl), kr = Pde::cell(a.pde, cr);
        const CT sl = Pde::speed(kl, qm, j), sr = Pde::speed(kr, qp, j);
        const CT sp = sl > sr ? sl : sr;
        CT Gv[V], Dq[V];
#pragma unroll
        for (int v = 0; v < V; v++) {
            Gv[v] = (CT)0.5 * (fm[v] + fp[v]) - (CT)0.5 * sp * (qp[v] - qm[v]);
            Dq[v] = (CT)0;
        }
        if constexpr (Pde::kNCP) {
            const CT deta = (qp[0] + qp[3]) - (qm[0] + qm[3]);
            Gv[0] = (CT)0.5 * (fm[0] + fp[0]) - (CT)0.5 * sp * deta;
            Gv[3] = (CT)0.5 * (fm[3] + fp[3]);
            Dq[1 + j] = (CT)0.5 * (CT)kl.g * (CT)0.5 * (qm[0] + qp[0]) * deta;
        }
#pragma unroll
        for (int v = 0; v < V; v++) {
            CT g = side ? Gv[v] + Dq[v] : Gv[v] - Dq[v];
            if constexpr (FP != P64) g = widen(round_to<FP>(g));
            G[(((cbi * DIM + j) * 2 + side) * V + v) * F + f] = g;
        }
    }
    __syncthreads();

    const int cb = tid / S, s = tid % S;
    const long cell = cell0 + cb;
    if (cb < CPB && cell < a.ncell) {
#pragma unroll
        for (int v = 0; v < V; v++) {
            double dq = 0.0;
#pragma unroll
            for (int j = 0; j < DIM; j++) {
                const int i = coord<n>(s, j);
                const int f = face_of<n, DIM>(s, j);
                const CT g0 = G[(((cb * DIM + j) * 2 + 0) * V + v) * F + f];
                const CT g1 = G[(((cb * DIM + j) * 2 + 1) * V + v) * F + f];
                if constexpr (FP == P64) {
                    dq += B->L0[i] * g0 - B->L1[i] * g1;
                } else {
                    dq += (double)(B->L0p[FP][i] * g0) - (double)(B->L1p[FP][i] * g1);
                }
            }
            double *qp_ = a.Q + (cell * V + v) * S + s;
            *qp_ = fma(a.sigma, dq, *qp_);
        }
    }
}

// ---------------------------------------------------------------------------
// Largest wave speed over all nodes and directions (for eq. CFL_condition).
// Non-negative doubles order like their bit patterns, so atomicMax on the
// 64-bit pattern gives the maximum.
// ---------------------------------------------------------------------------
template <class Pde, int DIM, int N>
__global__ __launch_bounds__(256) void k_maxeig(const double *Q, PdeArgs pde, long ncell,
                                                unsigned long long *out) {
    using Sh = Shape<DIM, N>;
    constexpr int S = Sh::S, V = Pde::V;
    __shared__ double red[256];
    double m = 0.0;
    const long total = ncell * S;
    for (long i = blockIdx.x * 256L + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
        const long c = i / S;
        const int s = i % S;
        double q[V];
#pragma unroll
        for (int v = 0; v < V; v++) q[v] = Q[(c * V + v) * S + s];
        const typename Pde::Coef k = Pde::cell(pde, c);
#pragma unroll
        for (int j = 0; j < DIM; j++) {
            const double l = Pde::speed(k, q, j);
            m = (l > m || l != l) ? l : m;
        }
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double o = red[threadIdx.x + w];
            const double x = red[threadIdx.x];
            red[threadIdx.x] = (o > x || o != o) ? o : x;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

}  // namespace aderdg
