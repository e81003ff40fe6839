// Host construction of the nodal basis and the ADER-DG operators in FP64
// (arXiv 2504.06889, Sec. 3), plus their roundings to each contraction format.
//
//  - Gauss-Legendre nodes/weights on [0,1] from the eigen-decomposition of the
//    Legendre Jacobi matrix (Golub-Welsch), by cyclic Jacobi rotations.
//  - Lagrange basis psi_k on the nodes (tensor-product basis of
//    eq. piecewise_solution); derivatives by the product rule.
//  - Time matrix of eq. Picard on [0,1]: K1[k][l] = psi_k(1) psi_l(1) -
//    int psi_k' psi_l; Picard operator Atau = K1^{-1} diag(w).
//  - Volume operator of eq. weak_form_volume_surface divided by the Gauss mass:
//    Kxi[k][l] = int psi_k' psi_l / w_k; face lifts L0 = psi(0)/w, L1 = psi(1)/w.
//  Integrals use an (n+1)-point Gauss rule, exact for these degrees.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "basis.h"

namespace aderdg {

// Symmetric eigenproblem by cyclic Jacobi rotations (A is overwritten; the
// eigenvectors are the columns of Z).
static void jacobi_eig(int n, std::vector<double> &A, std::vector<double> &Z) {
    Z.assign(n * n, 0.0);
    for (int i = 0; i < n; i++) Z[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0.0;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) off += A[p * n + q] * A[p * n + q];
        if (off < 1e-34) break;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) {
                const double apq = A[p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; k++) {  // columns p, q
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; k++) {  // rows p, q
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; k++) {
                    const double zkp = Z[k * n + p], zkq = Z[k * n + q];
                    Z[k * n + p] = c * zkp - s * zkq;
                    Z[k * n + q] = s * zkp + c * zkq;
                }
            }
    }
}

void gauss_legendre01(int n, double *x, double *w) {
    std::vector<double> J(n * n, 0.0), Z;
    for (int k = 1; k < n; k++) {
        const double b = k / std::sqrt(4.0 * k * k - 1.0);
        J[(k - 1) * n + k] = b;
        J[k * n + (k - 1)] = b;
    }
    jacobi_eig(n, J, Z);
    std::vector<int> idx(n);
    for (int i = 0; i < n; i++) idx[i] = i;
    for (int i = 0; i < n; i++)  // sort ascending by eigenvalue
        for (int j = i + 1; j < n; j++)
            if (J[idx[j] * n + idx[j]] < J[idx[i] * n + idx[i]]) std::swap(idx[i], idx[j]);
    for (int i = 0; i < n; i++) {
        const int e = idx[i];
        x[i] = 0.5 * (J[e * n + e] + 1.0);
        w[i] = Z[0 * n + e] * Z[0 * n + e];  // 2 v0^2 on [-1,1], halved on [0,1]
    }
}

static double lag(int n, const double *xi, int j, double x) {
    double v = 1.0;
    for (int m = 0; m < n; m++)
        if (m != j) v *= (x - xi[m]) / (xi[j] - xi[m]);
    return v;
}

static double lag_deriv(int n, const double *xi, int j, double x) {
    double sum = 0.0;
    for (int m = 0; m < n; m++) {
        if (m == j) continue;
        double term = 1.0 / (xi[j] - xi[m]);
        for (int p = 0; p < n; p++)
            if (p != j && p != m) term *= (x - xi[p]) / (xi[j] - xi[p]);
        sum += term;
    }
    return sum;
}

// Solve K X = B (n x n) by LU with partial pivoting, column by column.
static bool lu_solve(int n, const double *K, const double *Bm, double *X) {
    std::vector<double> A(K, K + n * n);
    std::vector<int> piv(n);
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
        if (A[p * n + c] == 0.0) return false;
        piv[c] = p;
        if (p != c)
            for (int k = 0; k < n; k++) std::swap(A[c * n + k], A[p * n + k]);
        for (int r = c + 1; r < n; r++) {
            A[r * n + c] /= A[c * n + c];
            for (int k = c + 1; k < n; k++) A[r * n + k] -= A[r * n + c] * A[c * n + k];
        }
    }
    for (int col = 0; col < n; col++) {
        std::vector<double> y(n);
        for (int i = 0; i < n; i++) y[i] = Bm[i * n + col];
        for (int c = 0; c < n; c++)
            if (piv[c] != c) std::swap(y[c], y[piv[c]]);
        for (int i = 0; i < n; i++)
            for (int k = 0; k < i; k++) y[i] -= A[i * n + k] * y[k];
        for (int i = n - 1; i >= 0; i--) {
            for (int k = i + 1; k < n; k++) y[i] -= A[i * n + k] * y[k];
            y[i] /= A[i * n + i];
        }
        for (int i = 0; i < n; i++) X[i * n + col] = y[i];
    }
    return true;
}

// Round-to-nearest-even to bfloat16 / binary16, returned as float.
float round_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return f;
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    float r;
    std::memcpy(&r, &u, 4);
    return r;
}

float round_fp16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t sign = u & 0x80000000u;
    uint32_t x = u ^ sign;
    if (x >= 0x7f800000u) return f;            // inf / nan
    float r;
    if (x >= 0x477ff000u) {                    // >= 65520 rounds to infinity
        x = 0x7f800000u;
    } else if (x < 0x38800000u) {              // below 2^-14: binary16 subnormals, step 2^-24
        float a;
        std::memcpy(&a, &x, 4);
        const float q = 5.9604644775390625e-8f;
        a = std::nearbyint(a / q) * q;
        std::memcpy(&x, &a, 4);
    } else {                                   // keep 10 explicit mantissa bits
        x += 0xfffu + ((x >> 13) & 1u);
        x &= 0xffffe000u;
    }
    x |= sign;
    std::memcpy(&r, &x, 4);
    return r;
}

float round_prec(int p, double v) {
    const float f = (float)v;
    if (p == 2) return round_bf16(f);
    if (p == 3) return round_fp16(f);
    return f;
}

bool build_basis(int n, DevBasis &B) {
    if (n < 1 || n > kMaxN) return false;
    std::memset(&B, 0, sizeof(B));
    double xi[kMaxN], w[kMaxN];
    gauss_legendre01(n, xi, w);
    double xq[kMaxN + 1], wq[kMaxN + 1];
    gauss_legendre01(n + 1, xq, wq);
    for (int i = 0; i < n; i++) {
        B.xi[i] = xi[i];
        B.w[i] = w[i];
        B.F0[i] = lag(n, xi, i, 0.0);
        B.F1[i] = lag(n, xi, i, 1.0);
        B.L0[i] = B.F0[i] / w[i];
        B.L1[i] = B.F1[i] / w[i];
        for (int k = 0; k < n; k++) B.D[i][k] = lag_deriv(n, xi, k, xi[i]);
    }
    // G[k][l] = int_0^1 psi_k' psi_l
    double G[kMaxN][kMaxN];
    for (int k = 0; k < n; k++)
        for (int l = 0; l < n; l++) {
            double s = 0.0;
            for (int m = 0; m <= n; m++) s += wq[m] * lag_deriv(n, xi, k, xq[m]) * lag(n, xi, l, xq[m]);
            G[k][l] = s;
        }
    std::vector<double> K1(n * n), W(n * n, 0.0), A(n * n);
    for (int k = 0; k < n; k++) {
        W[k * n + k] = w[k];
        for (int l = 0; l < n; l++) K1[k * n + l] = B.F1[k] * B.F1[l] - G[k][l];
    }
    if (!lu_solve(n, K1.data(), W.data(), A.data())) return false;
    for (int k = 0; k < n; k++) {
        double rs = 0.0;
        for (int l = 0; l < n; l++) {
            B.Atau[k][l] = A[k * n + l];
            B.Kxi[k][l] = G[k][l] / w[k];
            rs += A[k * n + l];
        }
        B.Arow[k] = rs;
    }
    for (int l = 0; l < n; l++) {
        double cs = 0.0;
        for (int k = 0; k < n; k++) cs += w[k] * A[k * n + l];
        B.wA[l] = cs;
    }
    for (int p = 0; p < 4; p++)
        for (int i = 0; i < n; i++) {
            B.F0p[p][i] = round_prec(p, B.F0[i]);
            B.F1p[p][i] = round_prec(p, B.F1[i]);
            B.L0p[p][i] = round_prec(p, B.L0[i]);
            B.L1p[p][i] = round_prec(p, B.L1[i]);
            for (int k = 0; k < n; k++) {
                B.Dp[p][i][k] = round_prec(p, B.D[i][k]);
                B.Kxip[p][i][k] = round_prec(p, B.Kxi[i][k]);
            }
        }
    return true;
}

double lagrange_value(int n, const double *xi, int j, double x) { return lag(n, xi, j, x); }

}  // namespace aderdg
