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


# ---- mixed-precision adjoint (predictor and volume formats below FP64) ----
# unit roundoff of each format (significant bits 24, 8, 11)
UNIT = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8, "fp16": 2.0 ** -11}
MIXED_PAIRS = [("fp32", "fp32"), ("bf16", "bf16"), ("fp16", "fp16"), ("fp16", "fp32"), ("fp32", "fp16")]


def _adjoint_pair(oracle_mod, dim, order, cells, prec, seed=1):
    """(FP64 adjoint, adjoint in prec, emulated forward J v in prec, FP64 J v, v, w)."""
    o = _oracle(oracle_mod, dim, order, cells)
    h = 1.0 / max(cells)
    e = oracle_mod.Oracle(dim, order, cells, (0.0,) * dim, tuple(c * h for c in cells), "acoustic",
                          (1.0, 2.25), prec=prec)
    c = inputs.lognormal_speed(o.ncell, seed=dim)
    o.set_material(c)
    e.set_material(c)
    dt = 0.3 * o.h / (dim * (2 * order + 1) * c.max())
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(o.shape)
    w = rng.standard_normal(o.shape)
    ref = o.adjoint_step(v, 0.0, dt, w, np.zeros(o.ncell))
    mix = e.adjoint_step(v, 0.0, dt, w, np.zeros(o.ncell))
    o.set_state(v)
    o.step(0.0, dt)
    e.set_state(v)
    e.step(0.0, dt)
    return ref, mix, e.get_state(), o.get_state(), v, w


@pytest.mark.parametrize("pp,pv", MIXED_PAIRS)
def test_mixed_adjoint_order0_is_exact(oracle_mod, pp, pv):
    """At N = 0 the derivative and volume matrices vanish: no transposed
    contraction carries anything, so the mixed adjoint equals the FP64 one bit
    for bit (a rounding anywhere else -- lam, mu, the face terms, the material
    derivative -- would show)."""
    (mu, g), (mup, gp), _, _, _, _ = _adjoint_pair(oracle_mod, 2, 0, (5, 4), (pp, pv, "fp64"))
    assert np.array_equal(mu, mup) and np.array_equal(g, gp)


@pytest.mark.parametrize("dim,order,cells", [(2, 3, (4, 3)), (3, 2, (3, 3, 2)), (3, 5, (2, 2, 2))])
@pytest.mark.parametrize("pp,pv", MIXED_PAIRS)
def test_mixed_adjoint_error_level(oracle_mod, dim, order, cells, pp, pv):
    """The mixed adjoint is the FP64 adjoint to the format's level: each
    transposed contraction is exact up to the rounding of its inputs (relative
    u each) and FP32 accumulation, and it moves mu = lam + O(sigma) terms by a
    fraction of that.  The error is not zero (the rounding happens) and stays
    below half a unit roundoff of the coarser format for mu, two units for the
    material derivative (a sum of products of two rounded quantities)."""
    (mu, g), (mup, gp), Jvp, Jv, v, w = _adjoint_pair(oracle_mod, dim, order, cells, (pp, pv, "fp64"))
    u = max(UNIT[pp], UNIT[pv])
    rm = np.linalg.norm(mup - mu) / np.linalg.norm(mu)
    rg = np.linalg.norm(gp - g) / np.linalg.norm(g)
    assert 1e-3 * u < rm < 0.5 * u, (rm, u)
    assert 1e-3 * u < rg < 2.0 * u, (rg, u)
    # dot-product test between the emulated forward and the emulated adjoint:
    # both are the exact operator to the format's level
    lhs, rhs = np.sum(w * Jvp), np.sum(mup * v)
    assert abs(lhs - rhs) <= 0.05 * u * np.linalg.norm(w) * np.linalg.norm(Jv), (lhs, rhs)


@pytest.mark.parametrize("dim,order,cells", [(2, 3, (4, 3)), (3, 2, (3, 3, 2))])
def test_mixed_adjoint_formats_go_to_their_contractions(oracle_mod, dim, order, cells):
    """Kxi^T acts on lam itself and reaches mu through the adjoint of the time
    average (first order in sigma); the transposed Picard derivatives act on
    that adjoint again (one more factor sigma ||D||).  So FP16 in the volume
    contraction moves mu more than FP16 in the predictor's: a swap of the two
    formats would reverse the order."""
    (mu, _), (m_pred16, _), _, _, _, _ = _adjoint_pair(oracle_mod, dim, order, cells, ("fp16", "fp32", "fp64"))
    (_, _), (m_vol16, _), _, _, _, _ = _adjoint_pair(oracle_mod, dim, order, cells, ("fp32", "fp16", "fp64"))
    e_pred = np.linalg.norm(m_pred16 - mu)
    e_vol = np.linalg.norm(m_vol16 - mu)
    assert e_pred < 0.5 * e_vol, (e_pred, e_vol)


@pytest.mark.parametrize("prec", [("fp16", "fp64", "fp64"), ("fp64", "fp16", "fp64"), ("fp16", "fp16", "fp16"),
                                  ("fp64", "fp64", "fp32")])
def test_mixed_adjoint_refuses_other_settings(oracle_mod, prec):
    """Predictor and volume both FP64 or both lower, flux FP64."""
    e = oracle_mod.Oracle(2, 3, (4, 3), (0.0, 0.0), (1.0, 0.75), "acoustic", (1.0, 2.25), prec=prec)
    e.set_material(np.ones(e.ncell))
    with pytest.raises(ValueError):
        e.adjoint_step(np.zeros(e.shape), 0.0, 1e-3, np.zeros(e.shape), np.zeros(e.ncell))


@pytest.mark.parametrize("pp,pv", [("fp16", "fp16"), ("bf16", "bf16"), ("fp16", "fp32")])
@pytest.mark.parametrize("k", [-40, -7, 30])
def test_mixed_adjoint_scale_invariant(oracle_mod, pp, pv, k):
    """The exact adjoint is linear in lam, so 2^k lam gives 2^k (mu, grad) bit
    for bit in FP64.  The mixed adjoint keeps that property through its
    per-cell power-of-two input scale: the rounded inputs are the same for
    every k, also where 2^k lam lies far below FP16's normal range (k = -40:
    values near 1e-12) and would otherwise underflow."""
    dim, order, cells = 3, 2, (3, 3, 2)
    h = 1.0 / max(cells)
    e = oracle_mod.Oracle(dim, order, cells, (0.0,) * dim, tuple(c * h for c in cells), "acoustic",
                          (1.0, 2.25), prec=(pp, pv, "fp64"))
    c = inputs.lognormal_speed(e.ncell, seed=4)
    e.set_material(c)
    dt = 0.3 * e.h / (dim * (2 * order + 1) * c.max())
    rng = np.random.default_rng(9)
    v = rng.standard_normal(e.shape)
    w = rng.standard_normal(e.shape)
    mu, g = e.adjoint_step(v, 0.0, dt, w, np.zeros(e.ncell))
    s = 2.0 ** k
    mus, gs = e.adjoint_step(v, 0.0, dt, s * w, np.zeros(e.ncell))
    assert np.array_equal(mus, s * mu) and np.array_equal(gs, s * g)
