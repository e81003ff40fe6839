"""Brute-force NumPy checks that pin the C oracle (test infrastructure only).

Each routine here is written from the paper's definitions by a different
route than ``aderdg_oracle.c``:

* ``dense_predictor``: the space-time system of eq. Picard for one cell of a
  linear, constant-coefficient PDE, assembled as Kronecker products of 1-D
  integrals computed exactly with ``numpy.polynomial`` (no Gauss rule, no
  Picard iteration) and solved with ``numpy.linalg.solve``.
* ``ck_time_average_1d``: the time average of the exact (Cauchy-Kowalevskaya /
  Taylor) solution of a 1-D linear system from polynomial data,
  sum_k (-dt A d/dx)^k / (k+1)! Q.
* ``fv_rusanov_step``: the textbook first-order Rusanov finite-volume update,
  which is what the scheme reduces to at N = 0.
* ``fv_swe_step``: the first-order path-conservative finite-volume update of
  the shallow-water system with the well-balanced Rusanov-type flux (eq.
  swe_custom_riemann), what the scheme reduces to at N = 0 for shallow water.
"""
import math

import numpy as np
from numpy.polynomial import legendre as npleg


def gl_nodes01(n):
    """Gauss-Legendre nodes and weights mapped to [0, 1] (library routine)."""
    x, w = npleg.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_polys(nodes):
    """Lagrange polynomials on `nodes` (in [0,1]) as Legendre series in y = 2x - 1
    (coefficients from the inverse Legendre-Vandermonde matrix, well conditioned
    at Gauss points)."""
    n = len(nodes)
    Vm = npleg.legvander(2.0 * np.asarray(nodes) - 1.0, n - 1)
    C = np.linalg.inv(Vm)          # column j: coefficients of psi_j
    return [C[:, j].copy() for j in range(n)]


def _val(c, x):
    return npleg.legval(2.0 * x - 1.0, c)


def nodal_basis_at(n, loc):
    """Tensor-product Lagrange basis on n Gauss-Legendre nodes per dimension at
    the reference point loc in [0,1]^d: phi[S] with node s = i0 + n i1 + ..."""
    xi, _ = gl_nodes01(n)
    ps = lagrange_polys(xi)
    out = np.ones(1)
    for x in loc:
        out = np.multiply.outer(np.array([_val(p, x) for p in ps]), out).reshape(-1)
    return out


def _der(c):
    return 2.0 * npleg.legder(c)   # d/dx = 2 d/dy


def _integrate01(c):
    ci = npleg.legint(c)
    return 0.5 * (npleg.legval(1.0, ci) - npleg.legval(-1.0, ci))


def one_d_integrals(n):
    """Exact 1-D integrals on [0,1]: mass M, derivative-test G[k][l] = int psi_k psi_l',
    and the time matrix T1[k][l] = psi_k(1) psi_l(1) - int psi_k' psi_l."""
    xi, _ = gl_nodes01(n)
    ps = lagrange_polys(xi)
    dps = [_der(p) for p in ps]
    mul = npleg.legmul
    M = np.array([[_integrate01(mul(ps[k], ps[l])) for l in range(n)] for k in range(n)])
    G = np.array([[_integrate01(mul(ps[k], dps[l])) for l in range(n)] for k in range(n)])
    T1 = np.array([[_val(ps[k], 1.0) * _val(ps[l], 1.0)
                    - _integrate01(mul(dps[k], ps[l])) for l in range(n)] for k in range(n)])
    F0 = np.array([_val(p, 0.0) for p in ps])
    return M, G, T1, F0, xi


def _kron_all(mats):
    out = np.ones((1, 1))
    for m in mats:
        out = np.kron(out, m)
    return out


def dense_predictor(Q, A_list, n, h, dt, source=None):
    """Exact solution of the cell-local space-time system of eq. Picard for a
    linear PDE q_t + sum_j A_j q_{x_j} = S with constant matrices A_j.

    Q: [V][S] nodal state (S = n^d, x fastest).  Returns q: [n][V][S], the
    space-time nodal values at the Gauss-Legendre time nodes.

    Weak form divided by h^d: (T1 (x) Ms) q + (dt/h) sum_j (Mt (x) Gj (x) M..) A_j q
    = (F0 (x) Ms) Q + dt (Mt (x) Ms) S, with all 1-D integrals exact.  `source`:
    None, or (var, phi[S], s[n]) for a source s(t_a) phi in the equation of
    variable `var`, given by its values at the space-time nodes (the point
    source of eq. exa_canonical_form projected onto the nodal basis)."""
    d = len(A_list)
    V = Q.shape[0]
    M, G, T1, F0, _ = one_d_integrals(n)
    # unknown ordering: (a, v, s) with s = i0 + n i1 + ..., i.e. kron order
    # (time) x (var) x (i_{d-1}) x ... x (i_0)
    def space_op(j, Mj):
        mats = []
        for dim in range(d - 1, -1, -1):
            mats.append(Mj if dim == j else M)
        return _kron_all(mats)
    Ms = space_op(-1, None)
    lhs = np.kron(T1, np.kron(np.eye(V), Ms))
    for j, A in enumerate(A_list):
        lhs = lhs + (dt / h) * np.kron(M, np.kron(A, space_op(j, G)))
    rhs = np.kron(F0[:, None], np.kron(np.eye(V), Ms)) @ Q.reshape(-1)
    if source is not None:
        var, phi, svals = source
        Sn = np.zeros((n, V, Q.shape[1]))
        Sn[:, var, :] = np.outer(svals, phi)
        rhs = rhs + dt * (np.kron(M, np.kron(np.eye(V), Ms)) @ Sn.reshape(-1))
    q = np.linalg.solve(lhs, rhs)
    return q.reshape(n, V, -1)


def ck_time_average_1d(Q, A, n, h, dt):
    """1-D: time average over [t, t+dt] of the exact solution from degree-N
    nodal data, sum_{k=0}^{N} (-dt A d/dx)^k / (k+1)! Q, with d/dx the exact
    derivative of the interpolating polynomial (built here from numpy's
    polynomial derivative, not from the oracle's matrix)."""
    xi, _ = gl_nodes01(n)
    ps = lagrange_polys(xi)
    # derivative matrix from exact polynomial derivatives
    Dm = np.array([[_val(_der(ps[j]), xi[i]) for j in range(n)] for i in range(n)])
    V = Q.shape[0]
    op = np.kron(A, Dm) / h  # acts on (v, s)
    term = Q.reshape(-1).copy()
    out = np.zeros_like(term)
    for k in range(n + V * n):  # series terminates (nilpotent); extra terms are exact zeros
        out += term / math.factorial(k + 1)
        term = -dt * (op @ term)
    return out.reshape(V, n)


def rusanov_flux(qm, qp, flux, speed):
    """Textbook Rusanov flux 0.5 (F(q-) + F(q+)) - 0.5 s (q+ - q-)."""
    s = np.maximum(speed(qm), speed(qp))
    return 0.5 * (flux(qm) + flux(qp)) - 0.5 * s * (qp - qm)


def fv_rusanov_step(U, dt, h, fluxes, speeds):
    """First-order finite volumes, periodic, with Rusanov fluxes.

    U: [V, C_{d-1}, ..., C_0] cell averages.  fluxes[j](U), speeds[j](U) act on
    arrays with the variable axis first."""
    d = U.ndim - 1
    out = U.copy()
    for j in range(d):
        ax = U.ndim - 1 - j            # array axis of dimension j
        Up = np.roll(U, -1, axis=ax)   # right neighbour
        G = rusanov_flux(U, Up, fluxes[j], speeds[j])   # flux at the right face
        Gm = np.roll(G, 1, axis=ax)                     # flux at the left face
        out = out - dt / h * (G - Gm)
    return out


def step_matrix(oracle, dt, t=0.0):
    """Assemble the (linear) one-step map of an oracle instance column by column."""
    N = oracle.ncell * oracle.V * oracle.S
    M = np.zeros((N, N))
    for i in range(N):
        e = np.zeros(N)
        e[i] = 1.0
        oracle.set_state(e.reshape(oracle.shape))
        oracle.step(t, dt)
        M[:, i] = oracle.get_state().reshape(-1)
    return M


def fv_swe_step(U, dt, h, g):
    """One first-order finite-volume step of the shallow-water system, periodic.

    U: [4, C_y, C_x] cell averages of (h, hu, hv, b).  Written from eq. swe_cons
    (fluxes (hu_j, hu u_j, hv u_j, 0)), eq. swe_noncons (the term g h d(h + b)/dx_j
    in the j-momentum) and eq. swe_custom_riemann: at every face between a left
    state L and a right state R along x_j, the conservative flux is the centred
    flux with a dissipation that acts on the surface eta = h + b and on the
    discharges, scaled by the largest characteristic speed |u_j| + sqrt(g h) of
    the two states; the non-conservative product along the straight path from L
    to R, g * (h_L + h_R)/2 * (eta_R - eta_L), is split in halves between the
    two cells.  With a piecewise-constant state the cell interiors contribute
    nothing, so the update is
        U_i <- U_i - dt/h [ (G + P/2)_{i+1/2} - (G - P/2)_{i-1/2} ]
    with G the flux and P the path integral (in the j-momentum only)."""
    out = U.copy()
    for j in range(2):
        ax = 2 - j                      # array axis of direction x_j (x fastest)
        L, R = U, np.roll(U, -1, axis=ax)   # the face on the right of each cell

        def flux(q):
            uj = q[1 + j] / q[0]
            return np.stack([q[1 + j], q[1] * uj, q[2] * uj, 0.0 * q[0]])

        def speed(q):
            return np.abs(q[1 + j] / q[0]) + np.sqrt(g * q[0])

        s = np.maximum(speed(L), speed(R))
        jump = np.stack([(R[0] + R[3]) - (L[0] + L[3]), R[1] - L[1], R[2] - L[2], 0.0 * L[0]])
        G = 0.5 * (flux(L) + flux(R)) - 0.5 * s * jump
        P = np.zeros_like(G)
        P[1 + j] = g * 0.5 * (L[0] + R[0]) * ((R[0] + R[3]) - (L[0] + L[3]))
        right = G + 0.5 * P                          # leaves cell i through its right face
        left = np.roll(G - 0.5 * P, 1, axis=ax)      # enters cell i through its left face
        out = out - dt / h * (right - left)
    return out


def fv_rusanov_step_typed(U, dt, h, flux, speed, xp, dtype):
    """First-order Rusanov finite volumes with every operation in one type:
    U[V, C0, C1] (periodic, already in `dtype`), flux(q, j) and speed(q, j) written
    with the array library `xp` (numpy, or torch for bfloat16) in that type.  The
    update visits the faces direction by direction, the lower face (side 0) before
    the upper one, each face flux G = 1/2 (F- + F+) - (1/2 s)(q+ - q-) with
    s = max(s-, s+), and adds +- sigma G: the order of operations of a kernel
    that computes in that type (the paper's semantics)."""
    half = xp.asarray(0.5, dtype=dtype) if xp is np else xp.tensor(0.5, dtype=dtype)
    sig = (np.float64(dt) / np.float64(h))
    sig = np.asarray(sig, dtype=dtype) if xp is np else xp.tensor(float(np.float32(sig)), dtype=dtype)
    out = U.copy() if xp is np else U.clone()
    for j in range(U.ndim - 1):
        ax = 1 + j
        for side in (0, 1):
            if side == 0:   # face between the left neighbour (-) and the cell (+)
                qm, qp = xp.roll(U, 1, ax) if xp is np else xp.roll(U, 1, ax), U
            else:           # face between the cell (-) and the right neighbour (+)
                qm, qp = U, (xp.roll(U, -1, ax) if xp is np else xp.roll(U, -1, ax))
            sm, sp_ = speed(qm, j), speed(qp, j)
            s = xp.maximum(sm, sp_)
            G = half * (flux(qm, j) + flux(qp, j)) - (half * s) * (qp - qm)
            t = sig * G
            out = out + t if side == 0 else out - t
    return out
