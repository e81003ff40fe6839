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
    double src_s[kMaxN];   // h s(t + xi_b dt) of the point source at the time nodes (host)
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

// In-place position-major FP64 line pass over the lines line_of(L), L < nl:
// X[i][line] <- sum_k M(i,k) X[k][line] with M(i,k) = T ? Mat[k][i] : Mat[i][k].
template <int n, bool T, class MT, class LineOf>
__device__ __forceinline__ void lines_inplace(double *X, int nl, int NLP, MT Mat, LineOf line_of, int tid,
                                              int nthreads) {
    for (int L = tid; L < nl; L += nthreads) {
        const int Ln = line_of(L);
        double x[n];
#pragma unroll
        for (int k = 0; k < n; k++) x[k] = X[k * NLP + Ln];
#pragma unroll
        for (int i = 0; i < n; i++) {
            double y = 0.0;
#pragma unroll
            for (int k = 0; k < n; k++) y = fma(T ? Mat[k][i] : Mat[i][k], x[k], y);
            X[i * NLP + Ln] = y;
        }
    }
}

// Line slots per direction j and cell: 0: F_j[0] = K v_j, 1: F_j[1+j] = p/rho
// (the only non-zero components of the acoustic flux), 2, 3: their
// K-tangents.  The adjoint passes use slots 0 and 1.
template <int DIM, int N>
struct AdjLayout {
    using Sh = Shape<DIM, N>;
    static constexpr int n = Sh::n, F = Sh::F, CPB = Sh::CPB, S = Sh::S;
    static constexpr int V = 1 + DIM;
    static constexpr int NZ = 4;
    static constexpr int NL = CPB * DIM * NZ * F;
    static constexpr int NLP = Fp64Pitch<n, DIM, NZ, CPB, Sh::TPB>::value;
    static constexpr size_t picard = (size_t)n * NLP * 8;
    static constexpr size_t faces = (size_t)2 * CPB * DIM * 2 * V * F * 8;  // q- and f-face adjoints
    // per-cell material-derivative terms, summed in a fixed order: one per face
    // node side (Rusanov speed) and one per thread (the rest)
    static constexpr int NRI = CPB * DIM * 2 * F;
    static constexpr size_t red = (size_t)(NRI + Sh::TPB) * 8;
    static constexpr size_t bytes = (picard > faces ? picard : faces) + red;
    // line of the L-th slot-0/1 line (L < CPB*DIM*2*F)
    __device__ static int half_line(int L) { return (L / (2 * F)) * (NZ * F) + L % (2 * F); }
};

template <int DIM, int N>
__global__ __launch_bounds__((Shape<DIM, N>::TPB)) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_adjoint(AdjKArgs a) {
    using Sh = Shape<DIM, N>;
    using AL = AdjLayout<DIM, N>;
    using Pde = Acoustic<DIM>;
    constexpr int n = Sh::n, S = Sh::S, F = Sh::F, CPB = Sh::CPB, TPB = Sh::TPB, V = 1 + DIM;
    constexpr int NLP = AL::NLP;
    __shared__ __attribute__((aligned(16))) char smem[AL::bytes];
    double *X = reinterpret_cast<double *>(smem);                                // [n][NLP]
    double *fbuf = reinterpret_cast<double *>(smem + AL::bytes - AL::red);  // [NRI] Rusanov-speed terms
    double *kbuf = fbuf + AL::NRI;                                           // [TPB] per-thread terms

    CBasis *B = (CBasis *)a.B;
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
    const double h = 1.0 / a.inv_h;
    const bool src_here = active && cell == a.src_cell;
    const double src_phi = src_here ? a.src_phi[s] : 0.0;
    const int iters = a.iters;

    // offset of this node on its line of each direction (slot 0)
    int po[DIM], pi[DIM], pf[DIM];
#pragma unroll
    for (int j = 0; j < DIM; j++) {
        pi[j] = coord<n>(s, j);
        pf[j] = face_of<n, DIM>(s, j);
        po[j] = pi[j] * NLP + ((cb * DIM + j) * AL::NZ) * F + pf[j];
    }
    constexpr int NHALF = CPB * DIM * 2 * F;  // slot 0/1 lines

    double Qn[V], lam[V];
#pragma unroll
    for (int v = 0; v < V; v++) {
        Qn[v] = active ? a.Qn[(cell * V + v) * S + s] : 0.0;
        lam[v] = active ? a.lam[(cell * V + v) * S + s] : 0.0;
    }

    // ---- forward Picard with its K-tangent ----
    // z[t] (zd[t]): the iterate (its K-derivative) at time node t; during an
    // iteration row b is reused for h R_b (h dR_b/dK) once slice b is done, and
    // after the last slice all rows become q_a = Q - sigma sum_b Atau[a][b] h R_b.
    // First iteration: all slices equal (Q, 0), one divergence serves them all.
    double z[n][V], zd[n][V];
#pragma unroll
    for (int t = 0; t < n; t++)
#pragma unroll
        for (int v = 0; v < V; v++) {
            z[t][v] = Qn[v];
            zd[t][v] = 0.0;
        }
    auto src_term = [&](int b) { return a.src_s[b] * src_phi; };
#pragma unroll 1
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int b = 0; b < n; b++) {
            if (it == 0 && b > 0) continue;
            if (slot) {
#pragma unroll
                for (int j = 0; j < DIM; j++) {
                    const double vj = z[b][1 + j], p = z[b][0], vdj = zd[b][1 + j], pd = zd[b][0];
                    X[po[j] + 0 * F] = active ? K * vj : 0.0;
                    X[po[j] + 1 * F] = active ? p * irho : 0.0;
                    X[po[j] + 2 * F] = active ? K * vdj + vj : 0.0;  // d(K v_j)/dK
                    X[po[j] + 3 * F] = active ? pd * irho : 0.0;
                }
            }
            __syncthreads();
            lines_inplace<n, false>(X, AL::NL, NLP, B->D, [](int L) { return L; }, tid, TPB);
            __syncthreads();
            if (active) {
                double r[V], rd[V];
                r[0] = 0.0;
                rd[0] = 0.0;
#pragma unroll
                for (int j = 0; j < DIM; j++) {
                    r[0] += X[po[j]];
                    rd[0] += X[po[j] + 2 * F];
                    r[1 + j] = X[po[j] + F];
                    rd[1 + j] = X[po[j] + 3 * F];
                }
                if (it == 0) {
#pragma unroll
                    for (int t = 0; t < n; t++) {
#pragma unroll
                        for (int v = 0; v < V; v++) {
                            double acc = B->Arow[t] * r[v];
                            if (v == 0 && src_here) {
#pragma unroll
                                for (int bb = 0; bb < n; bb++) acc = fma(B->Atau[t][bb], -src_term(bb), acc);
                            }
                            z[t][v] = fma(-a.sigma, acc, Qn[v]);
                            zd[t][v] = -a.sigma * (B->Arow[t] * rd[v]);
                        }
                    }
                } else {
                    if (src_here) r[0] -= src_term(b);
#pragma unroll
                    for (int t = 0; t < n; t++)
                        if (t == b) {
#pragma unroll
                            for (int v = 0; v < V; v++) {
                                z[t][v] = r[v];
                                zd[t][v] = rd[v];
                            }
                        }
                }
            }
        }
        if (it > 0 && active) {
#pragma unroll
            for (int v = 0; v < V; v++) {
                double r[n], rd[n];
#pragma unroll
                for (int b = 0; b < n; b++) {
                    r[b] = z[b][v];
                    rd[b] = zd[b][v];
                }
#pragma unroll
                for (int t = 0; t < n; t++) {
                    double acc = 0.0, accd = 0.0;
#pragma unroll
                    for (int b = 0; b < n; b++) {
                        acc = fma(B->Atau[t][b], r[b], acc);
                        accd = fma(B->Atau[t][b], rd[b], accd);
                    }
                    z[t][v] = fma(-a.sigma, acc, Qn[v]);
                    zd[t][v] = -a.sigma * accd;
                }
            }
        }
    }
    double qbar[V], qbard[V];
#pragma unroll
    for (int v = 0; v < V; v++) {
        qbar[v] = 0.0;
        qbard[v] = 0.0;
#pragma unroll
        for (int t = 0; t < n; t++) {
            qbar[v] = fma(B->w[t], z[t][v], qbar[v]);
            qbard[v] = fma(B->w[t], zd[t][v], qbard[v]);
        }
    }
    __syncthreads();

    // ---- adjoint of the face integral and the Rusanov flux, per face node ----
    double *gq = X;                                   // [cb][j][side][V][F]: adjoint of projected q
    double *gf = X + (size_t)CPB * DIM * 2 * V * F;   // adjoint of projected F_j . e_j
    {
        constexpr int NRI = AL::NRI;
        for (int itm = tid; itm < NRI; itm += TPB) {
            fbuf[itm] = 0.0;
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
            if (c_is_max) fbuf[itm] = sbar / (2.0 * rho * a.pde.mat[c]);
        }
    }
    __syncthreads();
    // expand the face adjoints into the cell (transpose of the projection); of
    // the flux adjoints only the components of F_j that are not identically
    // zero (0 and 1+j) are needed
    double qbb[V], fb0[DIM], fbj[DIM];
#pragma unroll
    for (int v = 0; v < V; v++) qbb[v] = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; j++) {
        fb0[j] = 0.0;
        fbj[j] = 0.0;
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
                if (v == 0) fb0[j] += e0 * gf[o0] + e1 * gf[o1];
                if (v == 1 + j) fbj[j] += e0 * gf[o0] + e1 * gf[o1];
            }
        }
    }
    __syncthreads();
    // volume integral adjoint: fbar_j += sigma Kxi^T (x)_j lam (components 0, 1+j)
    if (slot) {
#pragma unroll
        for (int j = 0; j < DIM; j++) {
            X[po[j]] = active ? lam[0] : 0.0;
            X[po[j] + F] = active ? lam[1 + j] : 0.0;
        }
    }
    __syncthreads();
    lines_inplace<n, true>(X, NHALF, NLP, B->Kxi, [](int L) { return AL::half_line(L); }, tid, TPB);
    __syncthreads();
    double kpart = 0.0;
    if (active) {
#pragma unroll
        for (int j = 0; j < DIM; j++) {
            fb0[j] += a.sigma * X[po[j]];
            fbj[j] += a.sigma * X[po[j] + F];
        }
        // fbar_j = A_j qbar: qbar_adj += A_j^T fbar_adj, and dK through A_j
#pragma unroll
        for (int j = 0; j < DIM; j++) {
            qbb[0] += fbj[j] * irho;
            qbb[1 + j] += K * fb0[j];
            kpart += fb0[j] * qbar[1 + j];
        }
#pragma unroll
        for (int v = 0; v < V; v++) kpart += qbb[v] * qbard[v];
    }

    // ---- transposed Picard iterations ----
    // rh[t]: adjoint of the iterate at time node t.  Each iteration first maps
    // the rows to Rbar_b = -dt sum_a Atau[a][b] rh_a, then slice b's row is
    // replaced by (1/h) sum_j D_j^T A_j^T Rbar_b once its lines are done.  First
    // iteration: rh_a = w_a qbb, so Rbar_b = wA[b] (-dt qbb) and one line pass
    // serves every slice.
    double mu[V], rh[n][V];
#pragma unroll
    for (int v = 0; v < V; v++) mu[v] = lam[v] + qbb[v];
    __syncthreads();
#pragma unroll 1
    for (int it = 0; it < iters; it++) {
        if (it > 0 && active) {
#pragma unroll
            for (int v = 0; v < V; v++) {
                double tmp[n];
#pragma unroll
                for (int t = 0; t < n; t++) tmp[t] = rh[t][v];
#pragma unroll
                for (int b = 0; b < n; b++) {
                    double r = 0.0;
#pragma unroll
                    for (int t = 0; t < n; t++) r = fma(B->Atau[t][b], tmp[t], r);
                    rh[b][v] = -a.dt * r;
                }
            }
        }
#pragma unroll
        for (int b = 0; b < n; b++) {
            if (it == 0 && b > 0) continue;
            double Rb[V];
#pragma unroll
            for (int v = 0; v < V; v++) Rb[v] = it == 0 ? -a.dt * qbb[v] : rh[b][v];
            if (slot) {
#pragma unroll
                for (int j = 0; j < DIM; j++) {
                    X[po[j]] = active ? Rb[1 + j] * irho : 0.0;
                    X[po[j] + F] = active ? K * Rb[0] : 0.0;
                }
            }
            __syncthreads();
            lines_inplace<n, true>(X, NHALF, NLP, B->D, [](int L) { return AL::half_line(L); }, tid, TPB);
            __syncthreads();
            if (active) {
                double nb_[V];
                nb_[0] = 0.0;
#pragma unroll
                for (int j = 0; j < DIM; j++) {
                    nb_[0] += X[po[j]];
                    nb_[1 + j] = X[po[j] + F];
                }
#pragma unroll
                for (int v = 0; v < V; v++) nb_[v] *= a.inv_h;
                if (it == 0) {
#pragma unroll
                    for (int bb = 0; bb < n; bb++)
#pragma unroll
                        for (int v = 0; v < V; v++) {
                            rh[bb][v] = B->wA[bb] * nb_[v];
                            mu[v] += rh[bb][v];
                        }
                } else {
#pragma unroll
                    for (int v = 0; v < V; v++) mu[v] += nb_[v];
#pragma unroll
                    for (int t = 0; t < n; t++)
                        if (t == b) {
#pragma unroll
                            for (int v = 0; v < V; v++) rh[t][v] = nb_[v];
                        }
                }
            }
        }
    }

    if (active) {
#pragma unroll
        for (int v = 0; v < V; v++) a.lam[(cell * V + v) * S + s] = mu[v];
    }
    // dJ/dc = dJ/dK * dK/dc: each cell's terms summed by one wavefront in a
    // fixed order (strided lane sums, then a butterfly), so the gradient is
    // reproducible bit for bit
    kbuf[tid] = active ? kpart : 0.0;
    __syncthreads();
    {
        const int lane = tid & 63, wave = tid >> 6;
        constexpr int FPC = DIM * 2 * F;  // face terms per cell
        for (int cr = wave; cr < CPB; cr += TPB / 64) {
            double acc = 0.0;
            for (int i = lane; i < FPC; i += 64) acc += fbuf[cr * FPC + i];
            for (int i = lane; i < S; i += 64) acc += kbuf[cr * S + i];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            const long c = cell0 + cr;
            if (lane == 0 && c < a.ncell) a.grad[c] += acc * 2.0 * rho * a.pde.mat[c];
        }
    }
}

}  // namespace aderdg
