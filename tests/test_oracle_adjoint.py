"""Pins of the oracle's discrete adjoint (acoustics with per-cell sound speed):
dot-product test of the step Jacobian, central finite differences of the
material derivative, and of the multi-step receiver misfit."""
import math

import numpy as np
import pytest

from oracle import misfit
from paper_2504_06889_amd import inputs


def _oracle(oracle_mod, dim=3, order=2, cells=(3, 3, 2), L=1.0):
    h = L / max(cells)
    return oracle_mod.Oracle(dim, order, cells, (0.0,) * dim, tuple(c * h for c in cells), "acoustic",
                             (1.0, 2.25))


@pytest.mark.parametrize("dim,order,cells", [(2, 3, (4, 3)), (3, 2, (3, 3, 2)), (3, 1, (2, 3, 4))])
def test_step_adjoint_dot_product(oracle_mod, dim, order, cells):
    o = _oracle(oracle_mod, dim, order, cells)
    rng = np.random.default_rng(dim + order)
    c = inputs.lognormal_speed(o.ncell, seed=dim)
    o.set_material(c)
    dt = 0.3 * o.h / (dim * (2 * order + 1) * c.max())
    v = rng.standard_normal(o.shape)
    w = rng.standard_normal(o.shape)
    o.set_state(v)
    o.step(0.0, dt)
    Jv = o.get_state()
    JTw, _ = o.adjoint_step(v, 0.0, dt, w, np.zeros(o.ncell))
    lhs, rhs = np.sum(w * Jv), np.sum(JTw * v)
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0) * 10, (lhs, rhs)


@pytest.mark.parametrize("dim,order,cells", [(2, 3, (4, 3)), (3, 2, (3, 3, 2))])
def test_material_derivative_central_differences(oracle_mod, dim, order, cells):
    o = _oracle(oracle_mod, dim, order, cells)
    rng = np.random.default_rng(7)
    c = inputs.lognormal_speed(o.ncell, seed=11)
    dt = 0.3 * o.h / (dim * (2 * order + 1) * c.max() * 1.2)
    Q = rng.standard_normal(o.shape)
    lam = rng.standard_normal(o.shape)
    o.set_material(c)
    _, g = o.adjoint_step(Q, 0.0, dt, lam, np.zeros(o.ncell))
    dc = rng.standard_normal(o.ncell)

    def obj(cc):
        o.set_material(cc)
        o.set_state(Q)
        o.step(0.0, dt)
        return float(np.sum(lam * o.get_state()))
    eps = 1e-6
    fd = (obj(c + eps * dc) - obj(c - eps * dc)) / (2 * eps)
    assert abs(fd - g @ dc) <= 1e-7 * max(abs(fd), 1e-12), (fd, g @ dc)


def test_misfit_gradient_central_differences_and_taylor(oracle_mod):
    """Multi-step misfit with a Ricker source and receivers: adjoint gradient vs
    central differences (1e-6 relative) and the Taylor remainder decaying as eps^2."""
    o = _oracle(oracle_mod, 3, 2, (4, 4, 4), L=2.0)
    c = inputs.lognormal_speed(o.ncell, mean=1.5, sigma=0.2, seed=0)
    xs = [1.0 + 0.1, 1.0 - 0.05, 1.0 + 0.02]
    o.set_source(xs, f0=5.0, t0=0.2, amp=1.0)
    rec = inputs.receivers_near(xs, o.h, nrec=8, half_cells=1.5, seed=1)
    dt = 0.5 * o.h / (3 * 5 * c.max())
    nsteps = 12
    Q0 = np.zeros(o.shape)
    # synthetic data from a homogeneous model
    _, data, _ = misfit.forward(o, Q0, np.full(o.ncell, 1.5), dt, nsteps, rec)
    J, g, _ = misfit.gradient(o, Q0, c, dt, nsteps, rec, data)
    assert J > 0
    dc = np.random.default_rng(3).standard_normal(o.ncell)

    def Jof(cc):
        return misfit.forward(o, Q0, cc, dt, nsteps, rec, data)[0]
    eps = 1e-6 * np.linalg.norm(c) / np.linalg.norm(dc)
    fd = (Jof(c + eps * dc) - Jof(c - eps * dc)) / (2 * eps)
    assert abs(fd - g @ dc) <= 1e-6 * abs(fd), (fd, g @ dc)
    # Taylor test: |J(c + e dc) - J(c) - e g.dc| = O(e^2)
    r = []
    for e in (1e-2, 5e-3, 2.5e-3):
        ee = e * np.linalg.norm(c) / np.linalg.norm(dc)
        r.append(abs(Jof(c + ee * dc) - J - ee * (g @ dc)))
    assert 3.0 < r[0] / r[1] < 5.0 and 3.0 < r[1] / r[2] < 5.0, r
