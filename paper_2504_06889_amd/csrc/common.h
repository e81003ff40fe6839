// Device-side building blocks of the ADER-DG step for gfx950 (MI355X):
// compile-time shapes, precision conversions, basis constants and the PDE
// systems of arXiv 2504.06889, Sec. 5.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace aderdg {

constexpr int kMaxN = 8;  // nodes per dimension supported (orders 0..7)

enum Prec { P64 = 0, P32 = 1, PBF16 = 2, PF16 = 3 };

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// ---------------------------------------------------------------------------
// Shapes and launch geometry for (DIM, N)
// ---------------------------------------------------------------------------
template <int DIM, int N>
struct Shape {
    static constexpr int n = N + 1;
    static constexpr int S = ipow(n, DIM);       // spatial nodes per cell
    static constexpr int F = ipow(n, DIM - 1);   // nodes per face
    // cells per workgroup: enough to fill >= 4 wavefronts of 64 lanes
    static constexpr int CPB = S >= 256 ? 1 : (256 / S);
    static constexpr int TPB = ((CPB * S + 63) / 64) * 64;
};

// ---------------------------------------------------------------------------
// Basis constants (built on the host in FP64 by basis.hip)
// ---------------------------------------------------------------------------
struct DevBasis {
    double xi[kMaxN], w[kMaxN];
    double D[kMaxN][kMaxN];     // D[i][k] = psi_k'(xi_i)
    double Atau[kMaxN][kMaxN];  // Picard time operator K1^{-1} W
    double Arow[kMaxN];         // row sums sum_b Atau[a][b] (equal to xi_a)
    double wA[kMaxN];           // weighted column sums sum_a w_a Atau[a][b]
    double Kxi[kMaxN][kMaxN];   // weak-form volume operator w_k' D[k'][k] / w_k
    double F0[kMaxN], F1[kMaxN];  // psi(0), psi(1)
    double L0[kMaxN], L1[kMaxN];  // face lifts psi(0)/w, psi(1)/w
    // the same operators rounded to each contraction format (index Prec; the
    // FP64 slot holds the FP32 rounding and is unused), stored as float
    float Dp[4][kMaxN][kMaxN];
    float Kxip[4][kMaxN][kMaxN];
    float F0p[4][kMaxN], F1p[4][kMaxN], L0p[4][kMaxN], L1p[4][kMaxN];
};

// Kernels read the basis through the constant address space: it does not
// change during a launch, so uniform reads become scalar loads.
using CBasis = const __attribute__((address_space(4))) DevBasis;

// The Picard time operator scaled by -sigma (sigma = dt/h) for one step size,
// formed on the device from the basis before the step's launches: the update
// q_a = Qn - sigma sum_b Atau[a][b] h R_b becomes one FMA chain from Qn.
struct ScaledTime {
    double At[kMaxN][kMaxN];  // -sigma Atau
    double Arow[kMaxN];       // -sigma Arow
    double wA[kMaxN];         // -sigma wA
};
using CScaled = const __attribute__((address_space(4))) ScaledTime;

// ---------------------------------------------------------------------------
// Precision conversions (round-to-nearest-even)
// ---------------------------------------------------------------------------
template <int P> struct Store;  // storage element of a contraction input
template <> struct Store<P64> { using T = double; };
template <> struct Store<P32> { using T = float; };
template <> struct Store<PBF16> { using T = __hip_bfloat16; };
template <> struct Store<PF16> { using T = _Float16; };

__device__ __forceinline__ double to_f(double x, double*) { return x; }

template <int P>
__device__ __forceinline__ typename Store<P>::T round_to(float x);
template <> __device__ __forceinline__ double round_to<P64>(float x) { return (double)x; }
template <> __device__ __forceinline__ float round_to<P32>(float x) { return x; }
template <> __device__ __forceinline__ __hip_bfloat16 round_to<PBF16>(float x) { return __float2bfloat16(x); }
template <> __device__ __forceinline__ _Float16 round_to<PF16>(float x) { return (_Float16)x; }

__device__ __forceinline__ float widen(float x) { return x; }
__device__ __forceinline__ float widen(__hip_bfloat16 x) { return __bfloat162float(x); }
__device__ __forceinline__ float widen(_Float16 x) { return (float)x; }
__device__ __forceinline__ double widen(double x) { return x; }

// Storage precision of the persistent state (Prec SP): each value is rounded
// to the format (FP32 first, then the format, nearest-even) whenever it is
// stored between traversals.
__device__ __forceinline__ double round_q(double x, int sp) {
    if (sp == P64) return x;
    const float f = (float)x;
    if (sp == P32) return (double)f;
    if (sp == PBF16) return (double)widen(round_to<PBF16>(f));
    return (double)widen(round_to<PF16>(f));
}

// The persistent state in HBM, element type by storage precision SP: FP64, or
// FP32/BF16/FP16 holding the value rounded as above.  Loads widen exactly to
// FP64 (all arithmetic stays FP64); stores round.  SP is uniform per launch.
__device__ __forceinline__ double load_state(const void *Q, long i, int sp) {
    if (sp == P64) return static_cast<const double *>(Q)[i];
    if (sp == P32) return (double)static_cast<const float *>(Q)[i];
    if (sp == PBF16) return (double)widen(static_cast<const __hip_bfloat16 *>(Q)[i]);
    return (double)widen(static_cast<const _Float16 *>(Q)[i]);
}
__device__ __forceinline__ void store_state(void *Q, long i, double x, int sp) {
    if (sp == P64) {
        static_cast<double *>(Q)[i] = x;
        return;
    }
    const float f = (float)x;
    if (sp == P32) static_cast<float *>(Q)[i] = f;
    else if (sp == PBF16) static_cast<__hip_bfloat16 *>(Q)[i] = round_to<PBF16>(f);
    else static_cast<_Float16 *>(Q)[i] = round_to<PF16>(f);
}
__host__ __device__ constexpr int state_bytes(int sp) { return sp == P64 ? 8 : (sp == P32 ? 4 : 2); }

// Face-value storage per FLUX precision
template <int P> struct FaceT { using T = typename Store<P>::T; };

// Component 1 + j of a state (the momentum in direction j) for a j that may be
// known only at run time: a select among the values, so that no register
// array is indexed dynamically.  The empty asm makes the three values opaque;
// otherwise the select of three loads is folded into one load through a
// computed index, which puts the array in scratch memory.
template <int DIM, class T>
__device__ __forceinline__ T mom(const T *q, int j) {
    if (__builtin_constant_p(j)) return q[1 + j];
    T a = q[1], b = q[2], c = q[DIM];
    asm("" : "+v"(a), "+v"(b), "+v"(c));
    return j == 0 ? a : ((DIM == 2 || j == 1) ? b : c);
}

// ---------------------------------------------------------------------------
// Per-cell physical parameters
// ---------------------------------------------------------------------------
struct PdeArgs {
    double prm[8];        // acoustic: rho, K | elastic: rho, lambda, mu | Euler: gamma | SWE: g
    const double *mat;    // per-cell sound speed (acoustic), or null
};

// ---------------------------------------------------------------------------
// PDE systems.  flux<T>(c, q, j, F): physical flux in direction j at one node;
// speed<T>(c, q, j): largest |eigenvalue| in direction j.  `c` is the
// per-cell coefficient block built by cell().
// ---------------------------------------------------------------------------
template <int DIM>
struct Acoustic {  // eq. acoustic: p_t + K div v = 0, rho v_t + grad p = 0
    static constexpr int V = 1 + DIM;
    static constexpr bool kNCP = false;
    static constexpr bool kLinear = true;
    static constexpr bool kPointSource = true;  // a point source may act on p
    struct Coef { double K, irho, c; };
    __device__ static Coef cell(const PdeArgs &a, long cell) {
        Coef c;
        double rho = a.prm[0];
        double sp = a.mat ? a.mat[cell] : sqrt(a.prm[1] / rho);
        c.K = rho * sp * sp;
        if (!a.mat) c.K = a.prm[1];
        c.irho = 1.0 / rho;
        c.c = sp;
        return c;
    }
    template <class T>
    __device__ static void flux(const Coef &c, const T *q, int j, T *F) {
        F[0] = (T)c.K * q[1 + j];
#pragma unroll
        for (int i = 0; i < DIM; i++) F[1 + i] = (i == j) ? q[0] * (T)c.irho : (T)0;
    }
    template <class T>
    __device__ static T speed(const Coef &c, const T *, int) { return (T)c.c; }
    // F_j[v] is identically zero unless v is p or v_j
    __host__ __device__ static constexpr bool flux_nz(int j, int v) { return v == 0 || v == 1 + j; }
};

template <int DIM>
struct Elastic {  // eq. equations_of_motion, q_t + A_j q_{x_j} = 0
    static constexpr int V = DIM * (DIM + 1) / 2 + DIM;
    static constexpr int NS = DIM * (DIM + 1) / 2;
    static constexpr bool kNCP = false;
    static constexpr bool kLinear = true;
    static constexpr bool kPointSource = false;
    struct Coef { double lam, mu, irho, cp; };
    __device__ static Coef cell(const PdeArgs &a, long) {
        Coef c;
        c.lam = a.prm[1];
        c.mu = a.prm[2];
        c.irho = 1.0 / a.prm[0];
        c.cp = sqrt((a.prm[1] + 2.0 * a.prm[2]) / a.prm[0]);
        return c;
    }
    __device__ static constexpr int sidx(int a, int b) {
        return a == b ? a
                      : (DIM == 2 ? 2
                                  : ((a + b == 1) ? 3 : ((a + b == 3) ? 4 : 5)));  // xy, yz, xz
    }
    template <class T>
    __device__ static void flux(const Coef &c, const T *q, int j, T *F) {
        const T *v = q + NS;
        const T lam = (T)c.lam, mu = (T)c.mu, ir = (T)c.irho;
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
            for (int b = a; b < DIM; b++) {
                const int k = sidx(a, b);
                if (a == b)
                    F[k] = -(a == j ? lam + (T)2 * mu : lam) * v[j];
                else
                    F[k] = (b == j) ? -mu * v[a] : ((a == j) ? -mu * v[b] : (T)0);
            }
#pragma unroll
        for (int i = 0; i < DIM; i++) F[NS + i] = -q[sidx(i, j)] * ir;
    }
    template <class T>
    __device__ static T speed(const Coef &c, const T *, int) { return (T)c.cp; }
    // F_j of a shear stress sigma_ab (a != b) is identically zero unless j is a or b
    __host__ __device__ static constexpr bool flux_nz(int j, int v) {
        if (v < DIM || v >= NS) return true;
        if (DIM == 2) return true;
        return v == 3 ? (j == 0 || j == 1) : (v == 4 ? (j == 1 || j == 2) : (j == 0 || j == 2));
    }
};

template <int DIM>
struct Euler {  // conserved (rho, rho v, E), ideal gas
    static constexpr int V = 2 + DIM;
    static constexpr bool kNCP = false;
    static constexpr bool kLinear = false;
    static constexpr bool kPointSource = false;
    struct Coef { double g; };
    __device__ static Coef cell(const PdeArgs &a, long) { return Coef{a.prm[0]}; }
    template <class T>
    __device__ static T pressure(const Coef &c, const T *q) {
        T ke = 0;
#pragma unroll
        for (int i = 0; i < DIM; i++) ke += q[1 + i] * q[1 + i];
        return ((T)c.g - (T)1) * (q[1 + DIM] - (T)0.5 * ke / q[0]);
    }
    template <class T>
    __device__ static void flux(const Coef &c, const T *q, int j, T *F) {
        const T p = pressure(c, q);
        const T mj = mom<DIM>(q, j);
        const T uj = mj / q[0];
        F[0] = mj;
#pragma unroll
        for (int i = 0; i < DIM; i++) F[1 + i] = q[1 + i] * uj + (i == j ? p : (T)0);
        F[1 + DIM] = uj * (q[1 + DIM] + p);
    }
    template <class T>
    __device__ static T speed(const Coef &c, const T *q, int j) {
        const T p = pressure(c, q);
        return fabs(mom<DIM>(q, j) / q[0]) + sqrt((T)c.g * p / q[0]);
    }
    __host__ __device__ static constexpr bool flux_nz(int, int) { return true; }
};

struct Swe {  // (h, hu, hv, b); pressure term as non-conservative g h grad(h+b)
    static constexpr int V = 4;
    static constexpr bool kNCP = true;
    static constexpr bool kLinear = false;
    static constexpr bool kPointSource = false;
    struct Coef { double g; };
    __device__ static Coef cell(const PdeArgs &a, long) { return Coef{a.prm[0]}; }
    template <class T>
    __device__ static void flux(const Coef &, const T *q, int j, T *F) {
        const T mj = mom<2>(q, j);
        const T uj = mj / q[0];
        F[0] = mj;
        F[1] = q[1] * uj;
        F[2] = q[2] * uj;
        F[3] = (T)0;
    }
    template <class T>
    __device__ static T speed(const Coef &c, const T *q, int j) {
        return fabs(mom<2>(q, j) / q[0]) + sqrt((T)c.g * q[0]);
    }
    // eta = h + b, whose reference derivative feeds the non-conservative term
    template <class T>
    __device__ static T ncp_input(const T *q) { return q[0] + q[3]; }
    // the bathymetry has no flux
    __host__ __device__ static constexpr bool flux_nz(int, int v) { return v < 3; }
};

// Flux in a direction j that is only known at run time (but uniform): one
// branch per direction, so that the PDE sees a compile-time j and no
// register array is indexed dynamically.
template <class Pde, int DIM, class T, class C>
__device__ __forceinline__ void flux_dir(const C &c, const T *q, int j, T *F) {
    if (j == 0) Pde::flux(c, q, 0, F);
    else if (DIM == 2 || j == 1) Pde::flux(c, q, 1, F);
    else Pde::flux(c, q, 2, F);
}

// ---------------------------------------------------------------------------
// Node index helpers (node = i0 + n i1 + n^2 i2)
// ---------------------------------------------------------------------------
template <int n>
__device__ __forceinline__ int coord(int s, int j) {
    return j == 0 ? s % n : (j == 1 ? (s / n) % n : s / (n * n));
}
template <int n>
__device__ __forceinline__ constexpr int stride(int j) {
    return j == 0 ? 1 : (j == 1 ? n : n * n);
}
// face node index of node s for direction j (coordinate j removed)
template <int n, int DIM>
__device__ __forceinline__ int face_of(int s, int j) {
    if (DIM == 2) return j == 0 ? s / n : s % n;
    if (j == 0) return s / n;
    if (j == 1) return (s % n) + n * (s / (n * n));
    return s % (n * n);
}
// first node of the line through face node f in direction j
template <int n>
__device__ __forceinline__ int line_start(int f, int j) {
    if (j == 0) return f * n;
    if (j == 1) return (f % n) + (f / n) * n * n;
    return f;
}

}  // namespace aderdg
