"""Pins of the oracle's Cauchy-Kowalevskaya predictor (linear PDEs), independent of
its own formula:
  - data that vary along x only make the cell-local problem one-dimensional, where
    d/dt = -A_x D_x / h maps degree-N polynomials to degree N-1: the exact local
    solution is a polynomial of degree N in time, which the space-time DG predictor
    reproduces exactly, so the converged Picard iteration (a separate code path)
    and the Taylor expansion agree at every time node;
  - the full CK scheme converges at order N+1 under refinement (planar wave);
  - the CK step stays close to the Picard step (both of order N+1);
  - nonlinear PDEs, point sources and the adjoint are refused."""
import math

import numpy as np
import pytest

from _util import small


def _oracle(oracle_mod, sc, predictor, iters=0, prec=("fp64",) * 3):
    return oracle_mod.Oracle(sc.dim, sc.order, sc.cells, sc.lo, sc.hi, sc.pde, sc.params,
                             picard_iters=iters, prec=prec, predictor=predictor)


CASES = [("acoustic", 2, 3, (1.0, 2.0), "planar_acoustic", {"k": (2 * math.pi, 0.0)}),
         ("acoustic", 3, 2, (1.0, 2.0), "planar_acoustic", {"k": (2 * math.pi, 0.0, 0.0)}),
         ("elastic", 2, 4, (1.0, 2.0, 1.0), "planar_elastic", {"kP": 2 * math.pi, "kS": 0.0}),
         ("elastic", 3, 3, (2.7, 32.4, 32.4), "planar_elastic", {"kP": 2 * math.pi, "kS": 0.0})]


@pytest.mark.parametrize("pde,dim,N,params,ic,extra", CASES)
def test_ck_equals_converged_picard_for_data_along_x(oracle_mod, pde, dim, N, params, ic, extra):
    cells = (3,) + (2,) * (dim - 1)
    sc = small(pde, dim, N, cells, (0.0,) * dim, tuple(c / 3.0 for c in cells), params, ic, extra)
    ck = _oracle(oracle_mod, sc, "ck")
    pc = _oracle(oracle_mod, sc, "picard", iters=6 * (N + 1))
    Q = sc.initial_state(ck.node_coords())
    rng = np.random.default_rng(4)
    # a random polynomial along x in each cell (same for every y, z), on top of the wave
    S, n = ck.S, ck.n
    ix = np.arange(S) % n
    Q = Q + rng.standard_normal((ck.ncell, ck.V, n))[:, :, ix]
    ck.set_state(Q)
    pc.set_state(Q)
    dt = 0.5 * ck.max_dt(0.5)
    for cell in (0, ck.ncell - 1):
        q1, b1, f1, _ = ck.predict_cell(cell, 0.0, dt)
        q2, b2, f2, _ = pc.predict_cell(cell, 0.0, dt)
        scale = np.abs(q2).max()
        np.testing.assert_allclose(q1, q2, rtol=0, atol=1e-11 * scale)
        np.testing.assert_allclose(b1, b2, rtol=0, atol=1e-11 * scale)
        np.testing.assert_allclose(f1, f2, rtol=0, atol=1e-11 * np.abs(f2).max())


def test_ck_converges_at_order_n_plus_1(oracle_mod):
    N = 2
    errs = []
    for C in (6, 12):
        sc = small("acoustic", 2, N, (C, C), (0.0, 0.0), (1.0, 1.0), (1.0, 1.0), "planar_acoustic",
                   {"k": (2 * math.pi, 2 * math.pi)})
        o = _oracle(oracle_mod, sc, "ck")
        X = o.node_coords()
        o.set_state(sc.initial_state(X))
        T = 0.1
        nst = int(math.ceil(T / o.max_dt(0.5)))
        A = o.run(nst, T / nst)
        errs.append(o.l2(A, sc.initial_state(X, T)))
    rate = math.log2(errs[0] / errs[1])
    assert rate > N + 1 - 0.4, (errs, rate)


@pytest.mark.parametrize("pde,dim,N,params,ic,extra", CASES[:1] + CASES[2:3])
def test_ck_step_close_to_picard_step(oracle_mod, pde, dim, N, params, ic, extra):
    two_pi = 2 * math.pi
    extra = {"k": (two_pi, two_pi)} if pde == "acoustic" else {"kP": two_pi, "kS": two_pi}
    sc = small(pde, dim, N, (5, 4), (0.0, 0.0), (1.0, 0.8), params, ic, extra)
    ck = _oracle(oracle_mod, sc, "ck")
    pc = _oracle(oracle_mod, sc, "picard")
    Q = sc.initial_state(ck.node_coords())
    ck.set_state(Q)
    pc.set_state(Q)
    dt = ck.max_dt(0.5)
    A = ck.run(3, dt)
    B = pc.run(3, dt)
    E = sc.initial_state(ck.node_coords(), 3 * dt)
    eA, eB = ck.l2(A, E), ck.l2(B, E)
    assert ck.l2(A, B) < 2 * max(eA, eB)
    assert eA < 3 * eB and eB < 3 * eA


def test_ck_refused_where_undefined(oracle_mod):
    sc = small("euler", 2, 2, (3, 3), (0.0, 0.0), (1.0, 1.0), (1.4,), "euler_density_wave")
    with pytest.raises(ValueError):
        _oracle(oracle_mod, sc, "ck")
    sc = small("acoustic", 2, 2, (3, 3), (0.0, 0.0), (1.0, 1.0), (1.0, 1.0), "zeros")
    o = _oracle(oracle_mod, sc, "ck")
    with pytest.raises(ValueError):
        o.set_source([0.5, 0.5], 5.0, 0.1)
