// HIP kernels of the ADER-DG time step (arXiv 2504.06889, Alg. 1) for gfx950.
//
//  k_predictor: one workgroup per CPB cells, one thread per spatial node.
//    Each thread keeps its node's space-time column (all time nodes, all
//    variables) in registers.  Per Picard iteration and time slice b the
//    pointwise fluxes F_j(q_b) are written to LDS, every 1-D line is
//    differentiated (D along x, y, z: in place on the vector ALU in FP64 or
//    FP32, or on the matrix cores in BF16/FP16 with FP32 accumulation), and the
//    owner thread folds the divergence into the FP64 Picard update
//    q_a <- Q - dt sum_b Atau[a][b] R_b (eq. Picard at the nodes); for a
//    linear PDE the Cauchy-Kowalevskaya procedure can replace the iteration
//    (N slices on the Taylor terms).  The epilogue forms the FP64 time
//    averages, projects them to the 2d faces (Alg. 1 "expansion") and adds
//    the volume integral to Q (on the matrix cores for linear PDEs in a
//    16-bit format).  The fused variant first runs the previous step's
//    corrector for its cells.
//  k_corrector: per cell, the Rusanov flux on each face node of its 2d faces
//    (eq. rusanov_flux; well-balanced form for shallow water) and the face
//    integral (lift) into Q in FP64.
//  Face buffer: faces[cell][dir][side][q|f][var][face node] in the FLUX format
//  (the f half is left unwritten where the corrector evaluates the flux from q).
#pragma once

#include <type_traits>

#include "common.h"

namespace aderdg {

struct StepArgs {
    void *Q;              // state [ncell][V][S] in the storage precision store_prec
    void *faces;          // face buffer written by the predictor
    const void *faces_in; // fused step: the previous step's face buffer (corrector input)
    const DevBasis *B;
    const ScaledTime *st; // the time operator scaled by -sigma for this dt
    PdeArgs pde;
    long ncell;
    int cells[3];
    double dt, inv_h, sigma, t, h;
    int vol_prec, flux_prec;
    int iters;            // Picard iterations
    int write_state;      // 0: only the face data is produced (Q untouched)
    int ck;               // 1: Cauchy-Kowalevskaya predictor (linear PDEs, no source)
    int store_prec;       // storage precision of Q (Prec): its element type; stored values are rounded to it
    long src_cell;        // -1: no source
    const double *src_phi;
    // point source: h s(t + xi_b dt) at the n time nodes and the time average
    // sum_b w_b s(t + xi_b dt) (uniform values, evaluated on the host)
    double src_s[kMaxN], src_bar;
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

// Periodic neighbour of a cell across its face in direction j (dir = +1 or
// -1).  Cell counts are below 2^31 (checked when a solver is created), so the
// index arithmetic is 32-bit.
__device__ __forceinline__ long neighbour(long cell, int j, int dir, const int *cells, int dim) {
    const unsigned c = (unsigned)cell, n0 = (unsigned)cells[0], n1 = (unsigned)cells[1], n2 = (unsigned)cells[2];
    unsigned x = c % n0, y = 0, z = 0;
    if (dim > 1) {
        const unsigned r = c / n0;
        y = r % n1;
        if (dim > 2) z = r / n1;
    }
    auto step = [dir](unsigned v, unsigned m) { return dir > 0 ? (v + 1 == m ? 0u : v + 1) : (v == 0 ? m - 1 : v - 1); };
    if (j == 0) x = step(x, n0);
    else if (j == 1) y = step(y, n1);
    else z = step(z, n2);
    return (long)(x + n0 * (y + n1 * z));
}

// ---------------------------------------------------------------------------
// FP64 line pass: X <- M along each line, in place (vector ALU).
// Lines are enumerated as (blk, f): blk indexes a block of S values, f the
// face node through which the line runs; the direction of block blk is
// dir_of(blk).
// ---------------------------------------------------------------------------
template <int n, int S, int F, class MT, class DirOf>
__device__ __forceinline__ void lines_fp64(double *X, int nblk, MT M, DirOf dir_of,
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

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two FP32 values rounded to nearest-even in a 16-bit format P and packed into
// one 32-bit word, the first in the low half (one conversion instruction).
template <int P>
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    if constexpr (P == PF16) return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, f16x2));
    else return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}

// ---------------------------------------------------------------------------
// Matrix-core derivative of variable pairs, inputs in format P (BF16 or FP16),
// FP32 accumulation.  Data: for every line pair LP (one line geometry,
// two variables), NPOS position slots (8, or 4 when n <= 4) x 2 variables,
// position pairs swizzled by the face node f of the line: element
// LP*2*NPOS + 4*((k/2) ^ sw(f)) + 2*(k%2) + var.  One 16x16 tile takes
// LPC = 8/NPOS line pairs per column of the B operand (K = (line pair,
// position, variable)); the constant A operand holds D on the interleaved
// block diagonal (row (line pair, i, var), column (line pair, k, var)), so a
// C column is the derivative of both variables of its line pairs.  FP32
// results go to Y[LP*OSTRIDE + 2*i + var] (OSTRIDE below).  Lane layouts (64
// lanes, 16x16x16): A[row = lane%16][k], B[k][col = lane%16],
// C[row = 4*(lane/16) + e][col], with lane group g = lane/16 holding
// k = 4g..4g+3.  The input swizzle spreads the owner writes over the LDS
// banks.  (FP32 contractions run on the vector ALU: the FP32 matrix cores take
// four 16x16x4 steps per tile on operands twice as wide.)
// ---------------------------------------------------------------------------
template <int n>
struct PairGeom {
    static constexpr int NPOS = n <= 4 ? 4 : 8;
    static constexpr int LPC = 8 / NPOS;   // line pairs per tile column
    static constexpr int PPL = NPOS / 2;   // position pairs per line
    static constexpr int LSTRIDE = 2 * NPOS;      // input elements per line pair
    // output floats per line pair, an odd number of float pairs (the 16 lanes
    // of a 64-bit store then cover the 32 banks once): all NPOS positions of
    // both variables.  Measured: not storing the padding rows costs 10 % (3-D
    // elastic N=5) although it saves LDS traffic.
    static constexpr int OSTRIDE = 2 * NPOS + 2;
    __device__ static constexpr int sw(int f) { return (f >> 2) & (PPL - 1); }
    __device__ static int in_off(int lp, int f, int k) { return lp * LSTRIDE + 4 * ((k >> 1) ^ sw(f)) + 2 * (k & 1); }
    __device__ static int out_off(int lp, int k) { return lp * OSTRIDE + 2 * k; }
};

template <int P, int n>
struct MfmaPairs {
    static_assert(P == PBF16 || P == PF16, "matrix-core pairs take a 16-bit format");
    using T = typename Store<P>::T;
    using VT = typename std::conditional<P == PBF16, i16x4, f16x4>::type;
    VT a;  // A operand

    using G = PairGeom<n>;
    template <class MT>
    __device__ void init(MT M, int lane) {
        const int r = lane & 15, g = lane >> 4;
        const int hr = r / G::LSTRIDE, i = (r % G::LSTRIDE) >> 1, vb = r & 1;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int k = 4 * g + e, hk = k / G::LSTRIDE, kp = (k % G::LSTRIDE) >> 1;
            const float val = (hr == hk && (k & 1) == vb && i < n && kp < n) ? M[i][kp] : 0.0f;
            if constexpr (P == PBF16) a[e] = __builtin_bit_cast(short, round_to<PBF16>(val));
            else a[e] = round_to<PF16>(val);
        }
    }

    template <int NTILE, int NWAVE, int F>
    __device__ void run(const T *X, float *Y, int wave, int lane) const {
        constexpr int TPW = (NTILE + NWAVE - 1) / NWAVE;
        constexpr int TB = TPW < 4 ? TPW : 4;
        constexpr bool EVEN = NTILE % NWAVE == 0;  // no tile guard per wavefront
        const int c = lane & 15, g = lane >> 4, gh = g / G::PPL, gp = g % G::PPL;
#pragma unroll
        for (int k0 = 0; k0 < TPW; k0 += TB) {
            f32x4 cc[TB];
            int lp[TB];
            VT bv[TB];
#pragma unroll
            for (int k = 0; k < TB; k++) {
                const int tile = wave + (k0 + k) * NWAVE;
                lp[k] = (tile * 16 + c) * G::LPC + gh;
                if (k0 + k < TPW && (EVEN || tile < NTILE))
                    bv[k] = *reinterpret_cast<const VT *>(X + lp[k] * G::LSTRIDE + 4 * (gp ^ G::sw(lp[k] % F)));
            }
#pragma unroll
            for (int k = 0; k < TB; k++) {
                const int tile = wave + (k0 + k) * NWAVE;
                if (k0 + k < TPW && (EVEN || tile < NTILE)) {
                    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
                    if constexpr (P == PBF16) cc[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv[k], z, 0, 0, 0);
                    else cc[k] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, bv[k], z, 0, 0, 0);
                }
            }
#pragma unroll
            for (int k = 0; k < TB; k++) {
                const int tile = wave + (k0 + k) * NWAVE;
                if (k0 + k < TPW && (EVEN || tile < NTILE)) {
                    float *y = Y + lp[k] * G::OSTRIDE + 4 * gp;
                    *reinterpret_cast<f32x2 *>(y) = f32x2{cc[k][0], cc[k][1]};
                    *reinterpret_cast<f32x2 *>(y + 2) = f32x2{cc[k][2], cc[k][3]};
                }
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Flux components that enter the Picard divergence: F_j[v] for the v whose
// flux is not identically zero in direction j, plus eta (index V) for the
// non-conservative term.  Lines of identically zero fluxes are skipped (their
// derivative is exactly zero).  The count is the same in every direction.
// ---------------------------------------------------------------------------
// eta for a system with a non-conservative term, else unused
template <class Pde, class T>
__device__ __forceinline__ T ncp_value(const T *q) {
    if constexpr (Pde::kNCP) return Pde::ncp_input(q);
    else return (T)0;
}

template <class Pde, int DIM>
struct FluxSupport {
    static constexpr int V = Pde::V;
    static constexpr int NV = Pde::kNCP ? V + 1 : V;
    __host__ __device__ static constexpr bool nz(int j, int v) { return v == V ? Pde::kNCP : Pde::flux_nz(j, v); }
    __host__ __device__ static constexpr int count(int j) {
        int c = 0;
        for (int v = 0; v < NV; v++) c += nz(j, v) ? 1 : 0;
        return c;
    }
    static constexpr int NZ = count(0);
    // component of the idx-th line of direction j (-1: padding)
    __host__ __device__ static constexpr int comp(int j, int idx) {
        int c = 0;
        for (int v = 0; v < NV; v++)
            if (nz(j, v)) {
                if (c == idx) return v;
                c++;
            }
        return -1;
    }
    // line index of component v in direction j (-1: identically zero)
    __host__ __device__ static constexpr int index(int j, int v) {
        if (!nz(j, v)) return -1;
        int c = 0;
        for (int u = 0; u < v; u++) c += nz(j, u) ? 1 : 0;
        return c;
    }
    // no direction before j has a nonzero F[v]: the divergence of v starts at j
    __host__ __device__ static constexpr bool first(int j, int v) {
        for (int u = 0; u < j; u++)
            if (nz(u, v)) return false;
        return true;
    }
    static constexpr bool same_count() {
        for (int j = 1; j < DIM; j++)
            if (count(j) != NZ) return false;
        return true;
    }
    static_assert(same_count(), "flux support must have the same size in every direction");
};

// ---------------------------------------------------------------------------
// Pitch of the FP64 position-major line buffer X[k][line], chosen at compile
// time among NL..NL+31 to minimise LDS bank conflicts of the owner accesses
// (lane t of the block touches X[k*P + line] with k, line from its node), under
// the bank model measured on gfx950: 64-bit writes are served 16 lanes at a
// time on 32 four-byte banks (conflict when two lanes' doubles agree mod 16),
// 64-bit reads 32 lanes at a time on 64 banks (doubles agree mod 32).  The
// line pass touches consecutive lines and is conflict-free for any pitch.
// ---------------------------------------------------------------------------
template <int n, int DIM, int NZ, int CPB, int TPB>
struct Fp64Pitch {
    static constexpr int S = ipow(n, DIM), F = ipow(n, DIM - 1), NL = CPB * DIM * NZ * F;
    struct Lanes {
        int k[TPB][DIM], base[TPB][DIM];  // k = -1: no node
    };
    static constexpr Lanes lanes() {
        Lanes L{};
        for (int t = 0; t < TPB; t++) {
            const int cb = t / S, s = t % S;
            for (int j = 0; j < DIM; j++) {
                const int crd = j == 0 ? s % n : (j == 1 ? (s / n) % n : s / (n * n));
                const int fce = DIM == 2 ? (j == 0 ? s / n : s % n)
                                         : (j == 0 ? s / n : (j == 1 ? (s % n) + n * (s / (n * n)) : s % (n * n)));
                L.k[t][j] = cb < CPB ? crd : -1;
                L.base[t][j] = (cb * DIM + j) * NZ * F + fce;
            }
        }
        return L;
    }
    static constexpr int cost(const Lanes &L, int P) {
        int c = 0;
        // every flux component shifts all lanes' lines by the same i*F, which
        // permutes the banks: the count is the same for each of the NZ components
        for (int w = 0; w < TPB / 64; w++)
            for (int j = 0; j < DIM; j++)
                for (int g = 0; g < 6; g++) {  // 4 write quarters (mod 16), 2 read halves (mod 32)
                    const int first = g < 4 ? 16 * g : 32 * (g - 4), len = g < 4 ? 16 : 32, mask = len - 1;
                    int cnt[32] = {};
                    int mx = 0;
                    for (int l = w * 64 + first; l < w * 64 + first + len; l++) {
                        if (L.k[l][j] < 0) continue;
                        const int b = (L.k[l][j] * P + L.base[l][j]) & mask;
                        mx = ++cnt[b] > mx ? cnt[b] : mx;
                    }
                    c += mx > 1 ? mx - 1 : 0;
                }
        return c * NZ;
    }
    static constexpr int best() {
        const Lanes L = lanes();
        int bp = NL | 1, bc = cost(L, NL | 1);
        for (int P = NL; P < NL + 32; P++) {
            const int c = cost(L, P);
            if (c < bc) {
                bc = c;
                bp = P;
            }
        }
        return bp;
    }
    static constexpr int value = best();
};
struct NoPitch {
    static constexpr int value = 1;
};

// Pitch of the FP32 line buffer: as for FP64 rows, but 32-bit reads and
// writes are served 32 lanes at a time on 32 four-byte banks (conflict when
// two lanes' floats agree mod 32).
template <int n, int DIM, int NZ, int CPB, int TPB>
struct Fp32Pitch {
    using P64 = Fp64Pitch<n, DIM, NZ, CPB, TPB>;
    static constexpr int NL = P64::NL;
    static constexpr int cost(const typename P64::Lanes &L, int P) {
        int c = 0;
        for (int w = 0; w < TPB / 64; w++)
            for (int j = 0; j < DIM; j++)
                for (int g = 0; g < 2; g++) {
                    int cnt[32] = {};
                    int mx = 0;
                    for (int l = w * 64 + 32 * g; l < w * 64 + 32 * g + 32; l++) {
                        if (L.k[l][j] < 0) continue;
                        const int b = (L.k[l][j] * P + L.base[l][j]) & 31;
                        mx = ++cnt[b] > mx ? cnt[b] : mx;
                    }
                    c += mx > 1 ? mx - 1 : 0;
                }
        return c;
    }
    static constexpr int best() {
        const typename P64::Lanes L = P64::lanes();
        int bp = NL | 1, bc = cost(L, NL | 1);
        for (int P = NL; P < NL + 32; P++) {
            const int c = cost(L, P);
            if (c < bc) {
                bc = c;
                bp = P;
            }
        }
        return bp;
    }
    static constexpr int value = best();
};

// ---------------------------------------------------------------------------
// Epilogue line buffers (face projection and volume integral), one direction
// at a time.  Input: position-major FP64 Ein[k][line] for the lines
// (cell, q|f, var, face node), odd pitch.  Volume output: FP64 Evol[i][line]
// for the lines (cell, var, face node).
// ---------------------------------------------------------------------------
template <class Pde, int DIM, int N>
struct EpiLayout {
    using Sh = Shape<DIM, N>;
    static constexpr int n = Sh::n, F = Sh::F, CPB = Sh::CPB, V = Pde::V;
    static constexpr int NLV = CPB * V * F;
    static constexpr int NLE = 2 * NLV;
    static constexpr int NLPE = NLE | 1, NLPV = NLV | 1;
    static constexpr size_t in_bytes = (size_t)n * NLPE * 8;
    static constexpr size_t bytes = in_bytes + (size_t)n * NLPV * 8;
};

// LDS of the predictor's phases other than the Picard lines: the epilogue,
// the non-conservative averages and the fused corrector.
template <class Pde, int DIM, int N>
struct RestLds {
    using Sh = Shape<DIM, N>;
    static constexpr size_t epi = EpiLayout<Pde, DIM, N>::bytes;
    static constexpr size_t ncp = Pde::kNCP ? (size_t)Sh::CPB * DIM * Sh::S * 8 : 0;
    static constexpr size_t corr = (size_t)Sh::CPB * DIM * 2 * Pde::V * Sh::F * 8;
    static constexpr size_t bytes = epi > ncp ? (epi > corr ? epi : corr) : (ncp > corr ? ncp : corr);
};

// Workgroups of up to four wavefronts that fit a CU's 160 KB of LDS (at most 3).
constexpr int lds_waves(size_t bytes) { return bytes * 3 <= 160 * 1024 ? 3 : (bytes * 2 <= 160 * 1024 ? 2 : 1); }

// ---------------------------------------------------------------------------
// Picard line buffers.
//  FP64 and FP32 (vector ALU): lines numbered ((cb*DIM + j)*NZ + i)*F + f
//        (block cell cb, direction j, i-th flux component of FluxSupport,
//        face node f), position-major X[k][line] with the bank-aware pitch NLP
//        (Fp64Pitch, Fp32Pitch), differentiated in place.
//  BF16/FP16 (matrix cores): line pairs LP = ((cb*DIM + j)*NP + p)*F + f for
//        the component pairs (2p, 2p+1) (an odd NZ is padded with a zero
//        component), in the MfmaPairs layout: the contraction format in, FP32
//        out.
// ---------------------------------------------------------------------------
template <class Pde, int DIM, int N, int PP>
struct PicardLayout {
    using Sh = Shape<DIM, N>;
    static constexpr int n = Sh::n, F = Sh::F, CPB = Sh::CPB;
    using FS = FluxSupport<Pde, DIM>;
    static constexpr int NZ = FS::NZ;
    // FP64 and FP32: the vector-ALU line pass
    static constexpr bool VALU = PP == P64 || PP == P32;
    static constexpr int NL = CPB * DIM * NZ * F;
    static constexpr int NLP =
        std::conditional<PP == P64, Fp64Pitch<n, DIM, NZ, CPB, Sh::TPB>,
                         typename std::conditional<PP == P32, Fp32Pitch<n, DIM, NZ, CPB, Sh::TPB>, NoPitch>::type>::type::value;
    __device__ static constexpr int elem(int line, int k) { return k * NLP + line; }
    static constexpr int VSTRIDE = F;
    // lower formats
    using G = PairGeom<n>;
    static constexpr int NP = (NZ + 1) / 2;
    static constexpr int NLPR = CPB * DIM * NP * F;
    static constexpr size_t esz = PP == P64 ? 8 : sizeof(typename Store<PP>::T);
    static constexpr size_t tile_bytes(int nt) {
        return (size_t)nt * 16 * 16 * esz + (size_t)nt * 16 * G::LPC * G::OSTRIDE * 4;
    }
    // Tiles: rounded up to a whole number per wavefront, so that the tile
    // loop needs no guard (the padding tiles read zeros and write outputs that
    // are never read), where that adds at most an eighth more tiles and keeps
    // the workgroups per CU; else the exact count.
    static constexpr int NWAVE = Sh::TPB / 64;
    static constexpr int NTILE0 = (NLPR + 16 * G::LPC - 1) / (16 * G::LPC);
    static constexpr int NTILEP = (NTILE0 + NWAVE - 1) / NWAVE * NWAVE;
    static constexpr size_t rest = RestLds<Pde, DIM, N>::bytes;
    static constexpr bool PAD =
        (NTILEP - NTILE0) * 8 <= NTILE0 &&
        lds_waves(tile_bytes(NTILEP) > rest ? tile_bytes(NTILEP) : rest) ==
            lds_waves(tile_bytes(NTILE0) > rest ? tile_bytes(NTILE0) : rest);
    static constexpr int NTILE = PAD ? NTILEP : NTILE0;
    static constexpr int PSTRIDE = G::LSTRIDE * F;   // input elements between variable pairs
    static constexpr int POSTRIDE = G::OSTRIDE * F;  // output floats between variable pairs
    static constexpr size_t in_bytes = (size_t)NTILE * 16 * 16 * esz;
    static constexpr size_t out_bytes = (size_t)NTILE * 16 * G::LPC * G::OSTRIDE * 4;
    static constexpr size_t bytes = VALU ? (size_t)n * NLP * (PP == P64 ? 8 : 4) : in_bytes + out_bytes;
};

// ---------------------------------------------------------------------------
// LDS budget of the predictor
// ---------------------------------------------------------------------------
template <class Pde, int DIM, int N, int PP>
struct PredLds {
    static constexpr size_t picard = PicardLayout<Pde, DIM, N, PP>::bytes;
    static constexpr size_t rest = RestLds<Pde, DIM, N>::bytes;
    static constexpr size_t bytes = picard > rest ? picard : rest;
};

// Target occupancy of the predictor (wavefronts per SIMD; a workgroup has at
// most four wavefronts, one per SIMD): three (at most 168 registers per lane)
// when the LDS holds three workgroups per CU, else two (256 registers) when it
// holds two.  The latency of the two barriers per slice needs the third
// wavefront: the FP64 3-D elastic order-5 kernel spills a few registers at
// this target (to scratch, outside the Picard loop) and still runs faster
// than at two.
template <class Pde, int DIM, int N, int PP>
struct PredOcc {
    static constexpr size_t lds = PredLds<Pde, DIM, N, PP>::bytes;
    static constexpr bool fits = Shape<DIM, N>::TPB <= 256;
    static constexpr int waves = !fits ? 1 : lds_waves(lds);
};

// For a linear flux with cell-constant coefficients and FP64 faces, the face
// projection of Fbar_j = F_j(qbar) equals F_j of the projected qbar, so only
// the projected qbar is stored and the corrector evaluates the flux from it
// (half the face traffic).
template <class Pde, int FP>
struct FluxFromFaceState {
    static constexpr bool value = Pde::kLinear && FP == P64;
};

// Projection of one line onto the face at side 0 (xi = 0) or 1 (xi = 1), as in
// Alg. 1 "expansion": FP64, or inputs rounded to the FLUX format FP and FP32
// accumulation; stored in the FLUX format.
template <int FP, int n>
__device__ __forceinline__ void project_store(void *faces, long idx, const double *x, CBasis *B, int side) {
    if constexpr (FP == P64) {
        double y = 0.0;
#pragma unroll
        for (int k = 0; k < n; k++) y = fma(side ? B->F1[k] : B->F0[k], x[k], y);
        reinterpret_cast<double *>(faces)[idx] = y;
    } else {
        float y = 0.0f;
#pragma unroll
        for (int k = 0; k < n; k++) y += (side ? B->F1p[FP][k] : B->F0p[FP][k]) * widen(round_to<FP>((float)x[k]));
        reinterpret_cast<typename FaceT<FP>::T *>(faces)[idx] = round_to<FP>(y);
    }
}

template <int P> struct PrecC { static constexpr int value = P; };

// ---------------------------------------------------------------------------
// Corrector of the block's cells (Alg. 1, second traversal): the Rusanov flux
// at every node of their 2d faces from `faces` (the cell's and its
// neighbours' face data, FLUX format FP), into the LDS array G, then per node
// the face integral (lift) added to Q*: qnew[v] = Q*[v] + sigma * lift.  The
// caller stores qnew (k_corrector) or keeps it as the next step's state
// (k_predictor, fused).  Threads of padding slots get qnew = 1.
template <class Pde, int DIM, int N, int FP>
__device__ __forceinline__ void correct_block(const StepArgs &a, const void *faces_v, char *smem, long cell0,
                                              int tid, double *qnew) {
    using Sh = Shape<DIM, N>;
    constexpr int n = Sh::n, S = Sh::S, F = Sh::F, CPB = Sh::CPB, TPB = Sh::TPB, V = Pde::V;
    using CT = typename std::conditional<FP == P64, double, float>::type;
    using FT = typename FaceT<FP>::T;
    CT *G = reinterpret_cast<CT *>(smem);  // [CPB][DIM][2][V][F]

    const DevBasis *B = a.B;
    const FT *faces = reinterpret_cast<const FT *>(faces_v);
    // this thread's node values of Q*, loaded first so that their latency
    // overlaps the Riemann solves
    const int cb = tid / S, s = tid % S;
    const long cell = cell0 + cb;
    const bool active = cb < CPB && cell < a.ncell;
    double qs[V];
#pragma unroll
    for (int v = 0; v < V; v++) qs[v] = active ? load_state(a.Q, (cell * V + v) * S + s, a.store_prec) : 1.0;

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
        const typename Pde::Coef kl = Pde::cell(a.pde, cl), kr = Pde::cell(a.pde, cr);
#pragma unroll
        for (int v = 0; v < V; v++) {
            qm[v] = (CT)widen(faces[bl + (long)v * F]);
            qp[v] = (CT)widen(faces[br + (long)v * F]);
        }
        if constexpr (FluxFromFaceState<Pde, FP>::value) {
            flux_dir<Pde, DIM>(kl, qm, j, fm);
            flux_dir<Pde, DIM>(kr, qp, j, fp);
        } else {
#pragma unroll
            for (int v = 0; v < V; v++) {
                fm[v] = (CT)widen(faces[bl + (long)(V + v) * F]);
                fp[v] = (CT)widen(faces[br + (long)(V + v) * F]);
            }
        }
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

#pragma unroll
    for (int v = 0; v < V; v++) {
        double dq = 0.0;
        if (active) {
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
        }
        // the corrected state as held in the storage precision (the fused kernel
        // keeps it in registers as the next step's state)
        qnew[v] = active ? round_q(fma(a.sigma, dq, qs[v]), a.store_prec) : 1.0;
    }
}

template <class Pde, int DIM, int N>
struct CorrLds {
    static constexpr size_t bytes = (size_t)Shape<DIM, N>::CPB * DIM * 2 * Pde::V * Shape<DIM, N>::F * 8;
};

template <class Pde, int DIM, int N, int FP>
__global__ __launch_bounds__((Shape<DIM, N>::TPB)) void k_corrector(StepArgs a) {
    using Sh = Shape<DIM, N>;
    constexpr int S = Sh::S, CPB = Sh::CPB, V = Pde::V;
    __shared__ __attribute__((aligned(16))) char smem[CorrLds<Pde, DIM, N>::bytes];
    const int tid = threadIdx.x;
    const long cell0 = xcd_block(blockIdx.x, gridDim.x) * CPB;
    double qnew[V];
    correct_block<Pde, DIM, N, FP>(a, a.faces, smem, cell0, tid, qnew);
    const int cb = tid / S, s = tid % S;
    const long cell = cell0 + cb;
    if (cb < CPB && cell < a.ncell) {
        for (int v = 0; v < V; v++) store_state(a.Q, (cell * V + v) * S + s, qnew[v], a.store_prec);
    }
}

// ---------------------------------------------------------------------------
// Predictor + face projection + volume integral (Alg. 1, first traversal)
// ---------------------------------------------------------------------------
// FUSE: first the corrector of the previous step for the block's cells (from
// a.faces_in and the Q* in a.Q), whose result is kept in registers as this
// step's state: one launch per step, and the memory-bound corrector of one
// workgroup overlaps the compute-bound predictor of another.
template <class Pde, int DIM, int N, int PP, bool FUSE>
__global__ __launch_bounds__((Shape<DIM, N>::TPB))
__attribute__((amdgpu_waves_per_eu(PredOcc<Pde, DIM, N, PP>::waves, 8))) void k_predictor(StepArgs a) {
    using Sh = Shape<DIM, N>;
    using L = PredLds<Pde, DIM, N, PP>;
    constexpr int n = Sh::n, S = Sh::S, F = Sh::F, CPB = Sh::CPB, TPB = Sh::TPB;
    constexpr int V = Pde::V;
    __shared__ __attribute__((aligned(16))) char smem[L::bytes];

    CBasis *B = (CBasis *)a.B;
    CScaled *ST = (CScaled *)a.st;
    // Issue priority: the wavefronts of a SIMD belong to different workgroups;
    // the phases bounded by barriers and memory latency (corrector, time
    // slices, epilogue) run at priority 2, the long FP64 Picard updates
    // (vector ALU only, no barrier) at 0, so that an update fills the issue
    // slots the other phases leave and does not delay a workgroup's barrier.
    __builtin_amdgcn_s_setprio(2);
    const int tid = threadIdx.x;
    const int cb = tid / S, s = tid % S;
    const long blk = xcd_block(blockIdx.x, gridDim.x);
    const long cell0 = blk * CPB;
    const long cell = cell0 + cb;
    const bool slot = cb < CPB;               // thread owns an LDS node slot
    const bool active = slot && cell < a.ncell;  // ... of a real cell
    const typename Pde::Coef coef = Pde::cell(a.pde, active ? cell : 0);

    double Qn[V];
    if constexpr (FUSE) {
        switch (a.flux_prec) {
        case P64: correct_block<Pde, DIM, N, P64>(a, a.faces_in, smem, cell0, tid, Qn); break;
        case P32: correct_block<Pde, DIM, N, P32>(a, a.faces_in, smem, cell0, tid, Qn); break;
        case PBF16: correct_block<Pde, DIM, N, PBF16>(a, a.faces_in, smem, cell0, tid, Qn); break;
        default: correct_block<Pde, DIM, N, PF16>(a, a.faces_in, smem, cell0, tid, Qn); break;
        }
        __syncthreads();  // the LDS is reused below
    } else {
#pragma unroll
        for (int v = 0; v < V; v++) Qn[v] = active ? load_state(a.Q, (cell * V + v) * S + s, a.store_prec) : 1.0;
    }

    // volume term of the node (sum over directions of Kxi along fbar_j)
    const int vp = a.vol_prec;
    double vol[V];
#pragma unroll
    for (int v = 0; v < V; v++) vol[v] = 0.0;
    bool vol_done = false;  // formed on the matrix cores with the predictor's buffers

    // (point sources act on acoustics only: for the other systems the source
    // terms are compiled out and hold no registers)
    const bool src_here = Pde::kPointSource && active && cell == a.src_cell;
    const double src_phi = src_here ? a.src_phi[s] : 0.0;
    const int iters = a.iters;

    // ---------------- Picard iterations (eq. Picard) ----------------
    // z[t] holds the FP64 iterate q_t at this node.  Within an iteration,
    // slice b's divergence only needs q_b, so once it is evaluated row b is
    // reused for h R_b (the 1/h of R_b is folded into sigma = dt/h); after the
    // last slice every row is replaced by q_a = Qn - sigma sum_b Atau[a][b] h R_b.
    // Per slice: the node owners write F_j(q_b) into the line buffer, every
    // line is differentiated, and the owners gather sum_j D_j F_j at their
    // node.  Each owner reads and writes only its own slots of the buffer,
    // which the line pass touches only between the two barriers, so two
    // barriers per slice suffice.
    // First iteration: every slice equals Qn, so slice 0's divergence serves
    // all of them: q_a = Qn - sigma (sum_b Atau[a][b]) h R_0 (+ source terms).
    // Padding cells (beyond ncell) hold Qn = 1 and never update it, so their
    // fluxes are finite: no stale or non-finite bits enter the lines.
    using PL = PicardLayout<Pde, DIM, N, PP>;
    // Lower-precision predictor of a linear system without non-conservative
    // term: the iterate is only ever used rounded to FP32 (flux input) or
    // through qbar (fbar = F(qbar)), and the FP32 divergence is exact in FP32,
    // so the rows can be FP32 with qbar accumulated in FP64 as the last
    // iterate is formed (same values as FP64 rows); the point source, an FP64
    // term, is then applied when the rows are combined.
    constexpr bool FR = PP != P64 && Pde::kLinear && !Pde::kNCP;
    using RowT = typename std::conditional<FR, float, double>::type;
    RowT z[n][V];
#pragma unroll
    for (int t = 0; t < n; t++)
#pragma unroll
        for (int v = 0; v < V; v++) z[t][v] = (RowT)Qn[v];
    double qbar[V];
#pragma unroll
    for (int v = 0; v < V; v++) qbar[v] = 0.0;
    // per-thread offset of its node in each direction's lines (variable 0)
    int po[DIM];
#pragma unroll
    for (int j = 0; j < DIM; j++) {
        const int f = face_of<n, DIM>(s, j), k = coord<n>(s, j);
        if constexpr (PL::VALU) po[j] = PL::elem(((cb * DIM + j) * PL::NZ) * F + f, k);
        else po[j] = ((cb * DIM + j) * PL::NP) * F + f;
    }
    auto src_term = [&](int b) {
        return a.src_s[b] * src_phi;
    };
    // fold h R_b (variable v, slice b) into the iterate rows; `last`: the
    // first iteration is also the last one
    auto fold = [&](int it, int b, int v, double r, bool last) __attribute__((always_inline)) {
        if (it == 0) {
#pragma unroll
            for (int t = 0; t < n; t++) {
                double qt = fma(ST->Arow[t], r, Qn[v]);
                if (v == 0 && src_here) {
#pragma unroll
                    for (int bb = 0; bb < n; bb++) qt = fma(ST->At[t][bb], -src_term(bb), qt);
                }
                if (FR && last) qbar[v] = fma(B->w[t], qt, qbar[v]);
                z[t][v] = (RowT)qt;
            }
        } else {
            if (!FR && v == 0 && src_here) r -= src_term(b);
#pragma unroll
            for (int bb = 0; bb < n; bb++)
                if (bb == b) z[bb][v] = (RowT)r;
        }
    };
    // end of an iteration > 0: rows hold h R_b; replace them by the new iterate.
    // After the last iteration of a linear system without non-conservative
    // term only the time average of the iterate is used (the flux average is
    // F_j(qbar)), and as the weights sum to one it is
    // sum_a w_a q_a = Qn - sigma sum_b wA[b] h R_b: n FMAs per variable
    // instead of n^2 + n (the same value up to FP64 rounding).
    constexpr bool QDIRECT = Pde::kLinear && !Pde::kNCP;
    auto update = [&](bool last) __attribute__((always_inline)) {
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int v = 0; v < V; v++) {
            double r[n];
#pragma unroll
            for (int b = 0; b < n; b++) {
                r[b] = (double)z[b][v];
                if (FR && v == 0 && src_here) r[b] -= src_term(b);
            }
            if (QDIRECT && last) {
                double acc = Qn[v];
#pragma unroll
                for (int b = 0; b < n; b++) acc = fma(ST->wA[b], r[b], acc);
                qbar[v] = acc;
                continue;
            }
#pragma unroll
            for (int t = 0; t < n; t++) {
                double acc = Qn[v];
#pragma unroll
                for (int b = 0; b < n; b++) acc = fma(ST->At[t][b], r[b], acc);
                z[t][v] = (RowT)acc;
            }
        }
        __builtin_amdgcn_s_setprio(2);
    };
    // Cauchy-Kowalevskaya procedure (linear flux, no source): the Taylor terms
    // T_k = dt^k/k! d^kq/dt^k from T_0 = Qn, T_k = -(sigma/k) h R(T_{k-1}),
    // k = 1..N, with h R the divergence of one slice; qbar = sum_k T_k/(k+1)
    // (FP64).  The terms only feed the next slice's flux and qbar.
    constexpr bool CKOK = Pde::kLinear && !Pde::kNCP;
    const bool ck = CKOK && a.ck;
    auto ck_run = [&](auto &&slice_fn) __attribute__((always_inline)) {
        double Tk[V];
#pragma unroll
        for (int v = 0; v < V; v++) {
            Tk[v] = Qn[v];
            qbar[v] = Qn[v];
        }
#pragma unroll 1
        for (int k = 1; k < n; k++) {
            const double sk = -a.sigma / k, ik = 1.0 / (k + 1);
            slice_fn(Tk, [&](int v, double r) __attribute__((always_inline)) {
                Tk[v] = sk * r;
                qbar[v] = fma(Tk[v], ik, qbar[v]);
            });
        }
    };
    if constexpr (PL::VALU) {
        // FP64, or FP32 (inputs rounded to FP32, FP32 accumulation, the sum
        // over the directions included; on the vector ALU, where the FP32
        // matrix cores' four 16x16x4 steps per tile and wide operands cost more)
        using XT = typename std::conditional<PP == P64, double, float>::type;
        XT *X = reinterpret_cast<XT *>(smem);  // [n][NLP] position-major
        // one slice: flux of the state q_b (rounded to XT) at every node into
        // the lines, the derivative along every line (in place), and the
        // divergence at the node passed to sink(v, h R_v) in descending v
        auto slice = [&](const auto *qrow, auto &&sink) __attribute__((always_inline)) {
            XT qb[V];
#pragma unroll
            for (int v = 0; v < V; v++) qb[v] = (XT)qrow[v];
            if (slot) {
#pragma unroll
                for (int j = 0; j < DIM; j++) {
                    XT Fv[V];
                    Pde::flux(coef, qb, j, Fv);
#pragma unroll
                    for (int i = 0; i < PL::NZ; i++) {
                        const int c = PL::FS::comp(j, i);
                        X[po[j] + i * PL::VSTRIDE] = c == V ? ncp_value<Pde>(qb) : Fv[c < V ? c : 0];
                    }
                }
            }
            __syncthreads();
            for (int Ln = tid; Ln < PL::NL; Ln += TPB) {
                XT x[n];
#pragma unroll
                for (int k = 0; k < n; k++) x[k] = X[k * PL::NLP + Ln];
#pragma unroll
                for (int i = 0; i < n; i++) {
                    XT y = 0;
#pragma unroll
                    for (int k = 0; k < n; k++) {
                        if constexpr (PP == P64) y = fma(B->D[i][k], x[k], y);
                        else y = fmaf(B->Dp[P32][i][k], x[k], y);
                    }
                    X[i * PL::NLP + Ln] = y;
                }
            }
            __syncthreads();
            if (active) {
                // descending v: the non-conservative term of v >= 1 reads q_b[0]
#pragma unroll
                for (int v = V - 1; v >= 0; v--) {
                    XT r = 0;
#pragma unroll
                    for (int j = 0; j < DIM; j++) {
                        const int i = PL::FS::index(j, v);
                        if (i >= 0) r += X[po[j] + i * PL::VSTRIDE];
                    }
                    double rr = (double)r;
                    if constexpr (Pde::kNCP) {
                        if (v >= 1 && v <= DIM) {
                            const XT eta = X[po[v - 1] + PL::FS::index(v - 1, V) * PL::VSTRIDE];
                            if constexpr (PP == P64) rr += coef.g * qb[0] * eta;
                            else rr += (double)((float)coef.g * qb[0] * eta);
                        }
                    }
                    sink(v, rr);
                }
            }
        };
        if (ck) {
            if constexpr (CKOK) ck_run(slice);
        } else {
            // the last update is peeled off the loop (it may form qbar directly)
            slice(z[0], [&](int v, double r) __attribute__((always_inline)) { fold(0, 0, v, r, iters == 1); });
#pragma unroll 1
            for (int it = 1; it < iters; it++) {
#pragma unroll
                for (int b = 0; b < n; b++)
                    slice(z[b], [&](int v, double r) __attribute__((always_inline)) { fold(it, b, v, r, false); });
                if (it < iters - 1 && active) update(false);
            }
            if (iters > 1 && active) update(true);
        }
    } else {
        using T = typename Store<PP>::T;
        T *Fb = reinterpret_cast<T *>(smem);
        float *Rb = reinterpret_cast<float *>(smem + PL::in_bytes);
        // zero the operand buffer once: padding positions, the padding variable
        // of an odd pair and the padding line pairs stay zero
        for (int i = tid; i < (int)(PL::in_bytes / 4); i += TPB) reinterpret_cast<uint32_t *>(smem)[i] = 0u;
        const int lane = tid & 63, wave = tid >> 6;
        constexpr int NWAVE = TPB / 64;
        MfmaPairs<PP, n> mp;
        mp.init(B->Dp[PP], lane);
        int io[DIM], oo[DIM];
#pragma unroll
        for (int j = 0; j < DIM; j++) {
            const int f = face_of<n, DIM>(s, j), k = coord<n>(s, j);
            io[j] = PL::G::in_off(po[j], f, k);
            oo[j] = PL::G::out_off(po[j], k);
        }
        __syncthreads();
        // One contraction pass on the matrix cores: the owners write the flux
        // components flux_j(j, Fv, eta) of every direction (rounded to the
        // format), M is applied along every line, and the owners sum their
        // node's results over the directions in FP32: sink(rf, eta) with rf[v]
        // the sum for variable v and eta[j] the derivative of the
        // non-conservative input along j.
        auto write_flux = [&](T *FbB, auto &&flux_j) __attribute__((always_inline)) {
#pragma unroll
            for (int j = 0; j < DIM; j++) {
                float Fv[V], ev;
                flux_j(j, Fv, ev);
                auto comp_val = [&](int c) -> float { return c < 0 ? 0.0f : (c == V ? ev : Fv[c < V ? c : 0]); };
#pragma unroll
                for (int p = 0; p < PL::NP; p++) {
                    T *dst = FbB + io[j] + p * PL::PSTRIDE;
                    const float f0 = comp_val(PL::FS::comp(j, 2 * p)), f1 = comp_val(PL::FS::comp(j, 2 * p + 1));
                    *reinterpret_cast<uint32_t *>(dst) = pack2<PP>(f0, f1);
                }
            }
        };
        auto gather = [&](const float *RbB, auto &&sink) __attribute__((always_inline)) {
            float rf[V], eta[DIM];
#pragma unroll
            for (int v = 0; v < V; v++) rf[v] = 0.0f;
#pragma unroll
            for (int j = 0; j < DIM; j++) {
#pragma unroll
                for (int p = 0; p < PL::NP; p++) {
                    const f32x2 r2 = *reinterpret_cast<const f32x2 *>(RbB + oo[j] + p * PL::POSTRIDE);
#pragma unroll
                    for (int h = 0; h < 2; h++) {
                        const int c = PL::FS::comp(j, 2 * p + h);
                        if (c >= 0 && c < V) {
                            if (PL::FS::first(j, c)) rf[c < V ? c : 0] = r2[h];
                            else rf[c < V ? c : 0] += r2[h];
                        }
                        if (Pde::kNCP && c == V) eta[j] = r2[h];
                    }
                }
            }
            if (active) sink(rf, eta);
        };
        auto pass = [&](const MfmaPairs<PP, n> &M, auto &&flux_j, auto &&sink) __attribute__((always_inline)) {
            if (slot) write_flux(Fb, flux_j);
            __syncthreads();
            M.template run<PL::NTILE, NWAVE, F>(Fb, Rb, wave, lane);
            __syncthreads();
            // every slot thread reads its results, so this block and the next
            // slice's flux writes share one condition; only real cells fold them
            if (slot) gather(Rb, sink);
        };
        // One slice: flux of q_b at every node, the derivative lines and the
        // divergence at the node, whose FP64 value for variable v goes to
        // sink(v, r) (descending v).  The flux sees the FP32 rounding of the
        // FP64 iterate (exact when FR).
        auto slice_flux = [&](const float *qb) __attribute__((always_inline)) {
            return [&, qb](int j, float *Fv, float &ev) __attribute__((always_inline)) {
                Pde::flux(coef, qb, j, Fv);
                ev = ncp_value<Pde>(qb);
            };
        };
        auto slice_sink = [&](const float *qb, auto &&sink) __attribute__((always_inline)) {
            return [&, qb](const float *rf, const float *eta) __attribute__((always_inline)) {
#pragma unroll
                for (int v = V - 1; v >= 0; v--) {
                    double rr = (double)rf[v];
                    if constexpr (Pde::kNCP) {
                        if (v >= 1 && v <= DIM) rr += (double)((float)coef.g * qb[0] * eta[v - 1]);
                    }
                    sink(v, rr);
                }
            };
        };
        auto slice = [&](int b, auto &&sink) __attribute__((always_inline)) {
            float qb[V];
#pragma unroll
            for (int v = 0; v < V; v++) qb[v] = (float)z[b][v];
            pass(mp, slice_flux(qb), slice_sink(qb, sink));
        };

        // The first and the last iteration are peeled off the loop, so that
        // qbar, formed with the last iterate, is not carried through it.
        if (ck) {
            if constexpr (CKOK)
                ck_run([&](const double *Tk, auto &&sink) __attribute__((always_inline)) {
                    float qb[V];
#pragma unroll
                    for (int v = 0; v < V; v++) qb[v] = (float)Tk[v];
                    pass(
                        mp,
                        [&](int j, float *Fv, float &ev) __attribute__((always_inline)) {
                            Pde::flux(coef, qb, j, Fv);
                            ev = 0.0f;
                        },
                        [&](const float *rf, const float *) __attribute__((always_inline)) {
#pragma unroll
                            for (int v = V - 1; v >= 0; v--) sink(v, (double)rf[v]);
                        });
                });
        } else if (iters == 1) {
            slice(0, [&](int v, double r) __attribute__((always_inline)) { fold(0, 0, v, r, true); });
        } else {
            slice(0, [&](int v, double r) __attribute__((always_inline)) { fold(0, 0, v, r, false); });
#pragma unroll 1
            for (int it = 1; it < iters; it++) {
#pragma unroll
                for (int b = 0; b < n; b++)
                    slice(b, [&](int v, double r) __attribute__((always_inline)) { fold(it, b, v, r, false); });
                if (it < iters - 1 && active) update(false);
            }
            if (active) update(true);
        }
        // Volume integral on the matrix cores when its format is the
        // predictor's 16-bit format (linear flux: fbar_j = F_j(qbar), FP64,
        // rounded to the format; Kxi in the format; FP32 accumulation, the sum
        // over the directions included).
        if constexpr (FR) {
            if (vp == PP) {
                MfmaPairs<PP, n> mk;
                mk.init(B->Kxip[PP], lane);
                pass(
                    mk,
                    [&](int j, float *Fv, float &ev) __attribute__((always_inline)) {
                        double Fd[V];
                        flux_dir<Pde, DIM>(coef, qbar, j, Fd);
#pragma unroll
                        for (int v = 0; v < V; v++) Fv[v] = (float)Fd[v];
                        ev = 0.0f;
                    },
                    [&](const float *rf, const float *) __attribute__((always_inline)) {
#pragma unroll
                        for (int v = 0; v < V; v++) vol[v] = (double)rf[v];
                    });
                vol_done = true;
            }
        }
    }
    __syncthreads();

    // ---------------- time averages (FP64) ----------------
    // qbar here; the flux averages fbar_j are formed per direction below
    double nbar[V];
#pragma unroll
    for (int v = 0; v < V; v++) {
        nbar[v] = 0.0;
        if constexpr (!FR) {
            // (formed by the last update when it was direct)
            if (!ck && !(QDIRECT && iters > 1)) {
#pragma unroll
                for (int t = 0; t < n; t++) qbar[v] = fma(B->w[t], z[t][v], qbar[v]);
            }
        }
    }
    if constexpr (Pde::kNCP) {
        // average of the non-conservative product: sum_a w_a g h_a D_j eta_a
        double *eb = reinterpret_cast<double *>(smem);  // [CPB][DIM][S]
#pragma unroll
        for (int t = 0; t < n; t++) {
            double qt[V];
#pragma unroll
            for (int v = 0; v < V; v++) qt[v] = z[t][v];
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
    // Per direction j: the owners write qbar and fbar_j at their position on
    // the lines along j; one thread per (cell, var, face node) projects both
    // lines onto the two faces (Alg. 1 "expansion") and, unless the matrix
    // cores already formed the volume term, applies Kxi along the fbar_j line
    // (FP64, or inputs rounded to the volume format with FP32 accumulation).
    // The owners then gather their node's volume term.  Two barriers per
    // direction: the line pass reads Ein and writes Evol, which the owners
    // only read after the second barrier and only overwrite (Ein) after it.
    // The fbar_j lines are skipped when neither the faces (q-only faces) nor
    // the volume term need them.
    using EL = EpiLayout<Pde, DIM, N>;
    double *Ein = reinterpret_cast<double *>(smem);                  // [n][NLPE]
    double *Evol = reinterpret_cast<double *>(smem + EL::in_bytes);  // [n][NLPV]
    const bool need_f = !vol_done || !(Pde::kLinear && a.flux_prec == P64);
    if (!need_f) {
        // Only the FP64 faces of qbar are left: one node-major copy of qbar
        // serves the lines of every direction, one pass and one barrier.
        double *Qb = reinterpret_cast<double *>(smem);  // [CPB][V][S]
        if (slot) {
#pragma unroll
            for (int v = 0; v < V; v++) Qb[(cb * V + v) * S + s] = active ? qbar[v] : 0.0;
        }
        __syncthreads();
        for (int L = tid; L < CPB * DIM * V * F; L += TPB) {
            const int f = L % F;
            int r = L / F;
            const int v = r % V;
            r /= V;
            const int j = r % DIM, cbi = r / DIM;
            const long c = cell0 + cbi;
            if (c >= a.ncell) continue;
            const int st = j == 0 ? 1 : (j == 1 ? n : n * n);
            const double *line = Qb + (cbi * V + v) * S + line_start<n>(f, j);
            double xq[n];
#pragma unroll
            for (int k = 0; k < n; k++) xq[k] = line[k * st];
            const long base = ((c * DIM + j) * 2) * 2 * V;
#pragma unroll
            for (int side = 0; side < 2; side++)
                project_store<P64, n>(a.faces, ((base + (side * 2 + 0) * V) + v) * (long)F + f, xq, B, side);
        }
    }
#pragma unroll 1
    for (int j = 0; j < (need_f ? DIM : 0); j++) {
        // fbar_j = sum_a w_a F_j(q_a); for a linear flux this is F_j(qbar)
        double fbj[V];
        if constexpr (Pde::kLinear) {
            flux_dir<Pde, DIM>(coef, qbar, j, fbj);
        } else {
#pragma unroll
            for (int v = 0; v < V; v++) fbj[v] = 0.0;
#pragma unroll
            for (int t = 0; t < n; t++) {
                double qt[V], Fv[V];
#pragma unroll
                for (int v = 0; v < V; v++) qt[v] = z[t][v];
                Pde::flux(coef, qt, j, Fv);
#pragma unroll
                for (int v = 0; v < V; v++) fbj[v] = fma(B->w[t], Fv[v], fbj[v]);
            }
        }
        const int ij = coord<n>(s, j), fj = face_of<n, DIM>(s, j);
        if (slot) {
#pragma unroll
            for (int v = 0; v < V; v++) {
                Ein[ij * EL::NLPE + ((cb * 2 + 0) * V + v) * F + fj] = active ? qbar[v] : 0.0;
                if (need_f) Ein[ij * EL::NLPE + ((cb * 2 + 1) * V + v) * F + fj] = active ? fbj[v] : 0.0;
            }
        }
        __syncthreads();
        auto line_pass = [&](auto fpc) {
            constexpr int FP = decltype(fpc)::value;
            for (int L = tid; L < EL::NLV; L += TPB) {
                const int f = L % F, r = L / F, v = r % V, cbi = r / V;
                const long c = cell0 + cbi;
                double xq[n], xf[n];
#pragma unroll
                for (int k = 0; k < n; k++) {
                    xq[k] = Ein[k * EL::NLPE + ((cbi * 2 + 0) * V + v) * F + f];
                    xf[k] = need_f ? Ein[k * EL::NLPE + ((cbi * 2 + 1) * V + v) * F + f] : 0.0;
                }
                if (c < a.ncell) {
                    const long base = ((c * DIM + j) * 2) * 2 * V;
#pragma unroll
                    for (int side = 0; side < 2; side++) {
                        project_store<FP, n>(a.faces, ((base + (side * 2 + 0) * V) + v) * (long)F + f, xq, B, side);
                        if (!FluxFromFaceState<Pde, FP>::value)
                            project_store<FP, n>(a.faces, ((base + (side * 2 + 1) * V) + v) * (long)F + f, xf, B,
                                                 side);
                    }
                }
                if (vol_done) continue;
                if (vp == P64) {
#pragma unroll
                    for (int i = 0; i < n; i++) {
                        double y = 0.0;
#pragma unroll
                        for (int k = 0; k < n; k++) y = fma(B->Kxi[i][k], xf[k], y);
                        Evol[i * EL::NLPV + L] = y;
                    }
                } else {
                    float xr[n];
#pragma unroll
                    for (int k = 0; k < n; k++) {
                        const float x = (float)xf[k];
                        xr[k] = vp == P32 ? x : (vp == PBF16 ? widen(round_to<PBF16>(x)) : widen(round_to<PF16>(x)));
                    }
#pragma unroll
                    for (int i = 0; i < n; i++) {
                        float y = 0.0f;
#pragma unroll
                        for (int k = 0; k < n; k++) y += B->Kxip[vp][i][k] * xr[k];
                        Evol[i * EL::NLPV + L] = (double)y;
                    }
                }
            }
        };
        switch (a.flux_prec) {
        case P64: line_pass(PrecC<P64>{}); break;
        case P32: line_pass(PrecC<P32>{}); break;
        case PBF16: line_pass(PrecC<PBF16>{}); break;
        default: line_pass(PrecC<PF16>{}); break;
        }
        __syncthreads();
        if (active && !vol_done) {
            const int l0 = (cb * V) * F + fj;
#pragma unroll
            for (int v = 0; v < V; v++) vol[v] += Evol[ij * EL::NLPV + l0 + v * F];
        }
    }

    if (active && a.write_state) {
        const double sbar = a.src_bar;
#pragma unroll
        for (int v = 0; v < V; v++) {
            double qn = Qn[v] + a.sigma * vol[v];
            if constexpr (Pde::kNCP) qn -= a.sigma * nbar[v];
            if (v == 0 && src_here) qn += a.dt * sbar * src_phi;
            store_state(a.Q, (cell * V + v) * S + s, qn, a.store_prec);  // Q* in the storage precision
        }
    }
}

// ---------------------------------------------------------------------------
// Largest wave speed over all nodes and directions (for eq. CFL_condition).
// Non-negative doubles order like their bit patterns, so atomicMax on the
// 64-bit pattern gives the maximum.
// ---------------------------------------------------------------------------
template <class Pde, int DIM, int N>
__global__ __launch_bounds__(256) void k_maxeig(const void *Q, int sp, PdeArgs pde, long ncell,
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
        for (int v = 0; v < V; v++) q[v] = load_state(Q, (c * V + v) * S + s, sp);
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
