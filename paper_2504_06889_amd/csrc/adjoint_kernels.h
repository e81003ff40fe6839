// Discrete adjoint of the ADER-DG step for linear acoustics with a per-cell
// sound speed c (bulk modulus K = rho c^2), FP64, gfx950.
//
// The step is affine in Q for a fixed material, so the adjoint of Q is the
// transpose of the step's linear part: face integral -> Rusanov flux -> face
// projection and volume integral -> time averages -> Picard iterations, in
// reverse order.  For linear fluxes the transposed Picard iteration is the
// Picard iteration with D -> D^T, Atau -> Atau^T and F_j -> A_j^T, so no
// forward iterate has to be stored.
//
// The material derivative of <lam, step(Q)> for cell c is computed in forward
// (tangent) mode: the predictor of cell c is differentiated with respect to
// K_c alongside its recomputation (dq/dK follows the same Picard iteration,
// driven by dF_j/dK = (v_j, 0, ..., 0)), and paired with the adjoints of the
// cell's time averages; the Rusanov speed s = max(c_L, c_R) adds
// -1/2 <G_adj, q+ - q-> ds/dK_c on each face where c is the larger speed
// (ties go to the left cell).
#pragma once

#include "kernels.h"

namespace aderdg {

struct AdjKArgs {
    const double *Qn;      // forward state at the step start
    double *lam;           // in: adjoint after the step; out: adjoint at the start
    double *grad;          // += d<lam, step>/dc per cell
    const double *lamface; // [cell][dir][side][V][F]: L_side^T contracted lam
    const double *fwdface; // forward face data of the step [cell][dir][side][q|f][V][F]
    const DevBasis *B;
    PdeArgs pde;
    long ncell;
    int cells[3];
    double dt, inv_h, sigma, t;
    int iters;
    long src_cell;
    const double *src_phi;
    double src_f0, src_t0, src_amp;
};

// lamface[c][j][side][v][f] = sum_i L_side[i] lam[c][v][node(f, j, i)]
template <int DIM, int N>
__global__ __launch_bounds__(256) void k_lamface(const double *lam, double *out, long ncell,
                                                 const DevBasis *B) {
    using Sh = Shape<DIM, N>;
    constexpr int n = Sh::n, S = Sh::S, F = Sh::F, V = 1 + DIM;
    const long total = ncell * DIM * 2 * V * F;
    for (long i = blockIdx.x * 256L + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
        const int f = i % F;
        long r = i / F;
        const int v = r % V;
        r /= V;
        const int side = r % 2;
        r /= 2;
        const int j = r % DIM;
        const long c = r / DIM;
        const int st = j == 0 ? 1 : (j == 1 ? n : n * n);
        const double *src = lam + (c * V + v) * S + line_start<n>(f, j);
        const double *L = side ? B->L1 : B->L0;
        double y = 0.0;
#pragma unroll
        for (int k = 0; k < n; k++) y = fma(L[k], src[k * st], y);
        out[i] = y;
    }
}

// Position-major FP64 line pass: Xout[i][L] = sum_k M(i,k) Xin[k][L] with
// M(i,k) = T ? Mat[k][i] : Mat[i][k].
template <int n, bool T>
__device__ __forceinline__ void lines_pm(const double *Xin, double *Xout, int NL, int NLP,
                                         const double (*Mat)[kMaxN], int tid, int nthreads) {
    for (int Ln = tid; Ln < NL; Ln += nthreads) {
        double x[n];
#pragma unroll
        for (int k = 0; k < n; k++) x[k] = Xin[k * NLP + Ln];
#pragma unroll
        for (int i = 0; i < n; i++) {
            double y = 0.0;
#pragma unroll
            for (int k = 0; k < n; k++) y = fma(T ? Mat[k][i] : Mat[i][k], x[k], y);
            Xout[i * NLP + Ln] = y;
        }
    }
}

template <int DIM, int N>
struct AdjLayout {
    using Sh = Shape<DIM, N>;
    static constexpr int n = Sh::n, F = Sh::F, CPB = Sh::CPB, S = Sh::S;
    static constexpr int V = 1 + DIM;
    static constexpr int NL = CPB * DIM * 2 * V * F;  // forward + tangent lines
    static constexpr int NLP = NL | 1;
    static constexpr size_t picard = (size_t)2 * n * NLP * 8;
    static constexpr size_t faces = (size_t)2 * CPB * DIM * 2 * V * F * 8;  // q- and f-face adjoints
    static constexpr size_t bytes = (picard > faces ? picard : faces) + (size_t)CPB * 8 * 4;
};

template <int DIM, int N>
__global__ __launch_bounds__((Shape<DIM, N>::TPB)) void k_adjoint(AdjKArgs a) {
    using Sh = Shape<DIM, N>;
    using AL = AdjLayout<DIM, N>;
    using Pde = Acoustic<DIM>;
    constexpr int n = Sh::n, S = Sh::S, F = Sh::F, CPB = Sh::CPB, TPB = Sh::TPB, V = 1 + DIM;
    constexpr int NLP = AL::NLP;
    __shared__ __attribute__((aligned(16))) char smem[AL::bytes];
    double *Xin = reinterpret_cast<double *>(smem);
    double *Xout = Xin + n * NLP;
    double *kred = reinterpret_cast<double *>(smem + AL::bytes - CPB * 8 * 4);  // per-cell partial sums

    const DevBasis *B = a.B;
    const int tid = threadIdx.x;
    const int cb = tid / S, s = tid % S;
    const long blk = xcd_block(blockIdx.x, gridDim.x);
    const long cell0 = blk * CPB;
    const long cell = cell0 + cb;
    const bool slot = cb < CPB;
    const bool active = slot && cell < a.ncell;
    const typename Pde::Coef coef = Pde::cell(a.pde, active ? cell : 0);
    const double rho = a.pde.prm[0];
    const double K = coef.K, irho = coef.irho;
    const bool src_here = active && cell == a.src_cell;
    const double src_phi = src_here ? a.src_phi[s] : 0.0;

    // offsets of this node on the lines of each direction (variable 0)
    int po[DIM], pi[DIM], pf[DIM];
#pragma unroll
    for (int j = 0; j < DIM; j++) {
        pi[j] = coord<n>(s, j);
        pf[j] = face_of<n, DIM>(s, j);
        po[j] = pi[j] * NLP + ((cb * DIM + j) * 2 * V) * F + pf[j];
    }

    double Qn[V], lam[V];
#pragma unroll
    for (int v = 0; v < V; v++) {
        Qn[v] = active ? a.Qn[(cell * V + v) * S + s] : 0.0;
        lam[v] = active ? a.lam[(cell * V + v) * S + s] : 0.0;
    }
    if (tid < CPB * 4) kred[tid] = 0.0;

    // ---- forward Picard with its K-tangent ----
    double q[n][V], qd[n][V], acc[n][V], accd[n][V];
#pragma unroll
    for (int t = 0; t < n; t++)
#pragma unroll
        for (int v = 0; v < V; v++) {
            q[t][v] = Qn[v];
            qd[t][v] = 0.0;
        }
#pragma unroll 1
    for (int it = 0; it < a.iters; it++) {
#pragma unroll
        for (int t = 0; t < n; t++)
#pragma unroll
            for (int v = 0; v < V; v++) {
                acc[t][v] = 0.0;
                accd[t][v] = 0.0;
            }
#pragma unroll 1
        for (int b = 0; b < n; b++) {
            double qb[V], qdb[V];
#pragma unroll
            for (int v = 0; v < V; v++) {
                qb[v] = q[0][v];
                qdb[v] = qd[0][v];
            }
#pragma unroll
            for (int t = 1; t < n; t++)
                if (t == b) {
#pragma unroll
                    for (int v = 0; v < V; v++) {
                        qb[v] = q[t][v];
                        qdb[v] = qd[t][v];
                    }
                }
            if (slot) {
#pragma unroll
                for (int j = 0; j < DIM; j++) {
                    double Fv[V], Fd[V];
                    Pde::flux(coef, qb, j, Fv);
                    Pde::flux(coef, qdb, j, Fd);
                    Fd[0] += qb[1 + j];  // dF_j/dK
#pragma unroll
                    for (int v = 0; v < V; v++) {
                        Xin[po[j] + v * F] = active ? Fv[v] : 0.0;
                        Xin[po[j] + (V + v) * F] = active ? Fd[v] : 0.0;
                    }
                }
            }
            __syncthreads();
            lines_pm<n, false>(Xin, Xout, AL::NL, NLP, B->D, tid, TPB);
            __syncthreads();
            if (active) {
                double R[V], Rd[V];
#pragma unroll
                for (int v = 0; v < V; v++) {
                    double r = 0.0, rd = 0.0;
#pragma unroll
                    for (int j = 0; j < DIM; j++) {
                        r += Xout[po[j] + v * F];
                        rd += Xout[po[j] + (V + v) * F];
                    }
                    R[v] = r * a.inv_h;
                    Rd[v] = rd * a.inv_h;
                }
                if (src_here) R[0] -= ricker(a.t + B->xi[b] * a.dt, a.src_f0, a.src_t0, a.src_amp) * src_phi;
#pragma unroll
                for (int t = 0; t < n; t++)
#pragma unroll
                    for (int v = 0; v < V; v++) {
                        acc[t][v] = fma(B->Atau[t][b], R[v], acc[t][v]);
                        accd[t][v] = fma(B->Atau[t][b], Rd[v], accd[t][v]);
                    }
            }
        }
#pragma unroll
        for (int t = 0; t < n; t++)
#pragma unroll
            for (int v = 0; v < V; v++) {
                q[t][v] = fma(-a.dt, acc[t][v], Qn[v]);
                qd[t][v] = -a.dt * accd[t][v];
            }
    }
    double qbar[V], qbard[V];
#pragma unroll
    for (int v = 0; v < V; v++) {
        qbar[v] = 0.0;
        qbard[v] = 0.0;
#pragma unroll
        for (int t = 0; t < n; t++) {
            qbar[v] = fma(B->w[t], q[t][v], qbar[v]);
            qbard[v] = fma(B->w[t], qd[t][v], qbard[v]);
        }
    }
    __syncthreads();

    // ---- adjoint of the face integral and the Rusanov flux, per face node ----
    double *gq = Xin;                                   // [cb][j][side][V][F]: adjoint of projected q
    double *gf = Xin + (size_t)CPB * DIM * 2 * V * F;   // adjoint of projected F_j . e_j
    {
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
            const double sl = a.pde.mat[cl], sr = a.pde.mat[cr];
            const double sp = sl >= sr ? sl : sr;
            const bool c_is_max = side ? (sl >= sr) : (sr > sl);
            double sbar = 0.0;
#pragma unroll
            for (int v = 0; v < V; v++) {
                const double lR = a.lamface[(((cr * DIM + j) * 2 + 0) * V + v) * (long)F + f];
                const double lL = a.lamface[(((cl * DIM + j) * 2 + 1) * V + v) * (long)F + f];
                const double G = a.sigma * (lR - lL);
                const double qm = a.fwdface[((((cl * DIM + j) * 2 + 1) * 2 + 0) * V + v) * (long)F + f];
                const double qp = a.fwdface[((((cr * DIM + j) * 2 + 0) * 2 + 0) * V + v) * (long)F + f];
                sbar += -0.5 * G * (qp - qm);
                const int o = (((cbi * DIM + j) * 2 + side) * V + v) * F + f;
                gq[o] = (side ? 0.5 : -0.5) * sp * G;
                gf[o] = 0.5 * G;
            }
            if (c_is_max) atomicAdd(&kred[cbi], sbar / (2.0 * rho * a.pde.mat[c]));
        }
    }
    __syncthreads();
    // expand the face adjoints into the cell (transpose of the projection)
    double qbb[V], fbb[DIM][V];
#pragma unroll
    for (int v = 0; v < V; v++) {
        qbb[v] = 0.0;
#pragma unroll
        for (int j = 0; j < DIM; j++) fbb[j][v] = 0.0;
    }
    if (active) {
#pragma unroll
        for (int j = 0; j < DIM; j++) {
            const double e0 = B->F0[pi[j]], e1 = B->F1[pi[j]];
#pragma unroll
            for (int v = 0; v < V; v++) {
                const int o0 = (((cb * DIM + j) * 2 + 0) * V + v) * F + pf[j];
                const int o1 = (((cb * DIM + j) * 2 + 1) * V + v) * F + pf[j];
                qbb[v] += e0 * gq[o0] + e1 * gq[o1];
                fbb[j][v] += e0 * gf[o0] + e1 * gf[o1];
            }
        }
    }
    __syncthreads();
    // volume integral adjoint: fbar_j += sigma Kxi^T (x)_j lam
    if (slot) {
#pragma unroll
        for (int j = 0; j < DIM; j++)
#pragma unroll
            for (int v = 0; v < V; v++) Xin[po[j] + v * F] = active ? lam[v] : 0.0;
    }
    __syncthreads();
    lines_pm<n, true>(Xin, Xout, AL::NL, NLP, B->Kxi, tid, TPB);
    __syncthreads();
    double kpart = 0.0;
    if (active) {
#pragma unroll
        for (int j = 0; j < DIM; j++)
#pragma unroll
            for (int v = 0; v < V; v++) fbb[j][v] += a.sigma * Xout[po[j] + v * F];
        // fbar_j = A_j qbar: qbar_adj += A_j^T fbar_adj, and dK through A_j
#pragma unroll
        for (int j = 0; j < DIM; j++) {
            qbb[0] += fbb[j][1 + j] * irho;
            qbb[1 + j] += K * fbb[j][0];
            kpart += fbb[j][0] * qbar[1 + j];
        }
#pragma unroll
        for (int v = 0; v < V; v++) kpart += qbb[v] * qbard[v];
    }

    // ---- transposed Picard iterations ----
    double mu[V];
    double rh[n][V];  // adjoint of the current iterate, per time node
#pragma unroll
    for (int v = 0; v < V; v++) mu[v] = lam[v] + qbb[v];
#pragma unroll
    for (int t = 0; t < n; t++)
#pragma unroll
        for (int v = 0; v < V; v++) rh[t][v] = B->w[t] * qbb[v];
    __syncthreads();
#pragma unroll 1
    for (int it = 0; it < a.iters; it++) {
        double rn[n][V];
#pragma unroll
        for (int t = 0; t < n; t++)
#pragma unroll
            for (int v = 0; v < V; v++) rn[t][v] = 0.0;
#pragma unroll 1
        for (int b = 0; b < n; b++) {
            // Rbar_b = -dt sum_a Atau[a][b] rh_a, then A_j^T per direction
            double Rb[V];
#pragma unroll
            for (int v = 0; v < V; v++) {
                double r = 0.0;
#pragma unroll
                for (int t = 0; t < n; t++) r = fma(B->Atau[t][b], rh[t][v], r);
                Rb[v] = -a.dt * r;
            }
            if (slot) {
#pragma unroll
                for (int j = 0; j < DIM; j++) {
#pragma unroll
                    for (int v = 0; v < V; v++) Xin[po[j] + v * F] = 0.0;
                    Xin[po[j] + 0 * F] = active ? Rb[1 + j] * irho : 0.0;
                    Xin[po[j] + (1 + j) * F] = active ? K * Rb[0] : 0.0;
                }
            }
            __syncthreads();
            lines_pm<n, true>(Xin, Xout, AL::NL, NLP, B->D, tid, TPB);
            __syncthreads();
            double nb_[V];
#pragma unroll
            for (int v = 0; v < V; v++) {
                double r = 0.0;
                if (slot) {
#pragma unroll
                    for (int j = 0; j < DIM; j++) r += Xout[po[j] + v * F];
                }
                nb_[v] = r * a.inv_h;
                mu[v] += nb_[v];
            }
#pragma unroll
            for (int t = 0; t < n; t++)
                if (t == b) {
#pragma unroll
                    for (int v = 0; v < V; v++) rn[t][v] = nb_[v];
                }
        }
#pragma unroll
        for (int t = 0; t < n; t++)
#pragma unroll
            for (int v = 0; v < V; v++) rh[t][v] = rn[t][v];
    }

    if (active) {
#pragma unroll
        for (int v = 0; v < V; v++) a.lam[(cell * V + v) * S + s] = mu[v];
    }
    // dJ/dc = dJ/dK * dK/dc, reduced over the cell's threads
    __syncthreads();
    if (active) atomicAdd(&kred[cb], kpart);
    __syncthreads();
    if (slot && s == 0 && active) {
        const double c = a.pde.mat[cell];
        a.grad[cell] += kred[cb] * 2.0 * rho * c;
    }
}

}  // namespace aderdg
