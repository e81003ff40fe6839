"""Pins of the oracle's shallow-water flow terms and of its 3-D elastic system.

* Shallow water (Sec. 5.4, eq. swe_cons, eq. swe_noncons, eq.
  swe_custom_riemann): at N = 0 the step must be the first-order
  path-conservative finite-volume update written out independently in
  ``oracle/brute.py`` (flowing states over a varying bottom, so the momentum
  flux, the wave speed, the surface dissipation and the split of the
  non-conservative product all carry weight), and at N >= 1 the scheme must
  converge at order N + 1 to a small gravity wave riding on a uniform stream
  (the momentum-flux Jacobian and the volume term g h d(h + b)/dx_j both enter
  the linearised dynamics).
* 3-D elastic waves (Sec. 5.2, eq. equations_of_motion and eq.
  elastic_matrices extended to three dimensions): convergence at order N + 1
  to superposed P and S plane waves along an oblique wave vector, which move
  every stress and velocity component with distinct values; the closed form
  is itself checked against the paper's printed 2-D matrices.
"""
import math

import numpy as np
import pytest

from oracle import brute
from paper_2504_06889_amd import inputs
from _util import make_oracle, paper_matrix, small


def _error_at(oracle_mod, sc, cells, T):
    o = make_oracle(oracle_mod, sc, cells)
    o.set_state(sc.initial_state(o.node_coords(), 0.0))
    nsteps = int(math.ceil(T / o.max_dt(sc.cfl)))
    Q = o.run(nsteps, T / nsteps)
    return o.l2(Q, sc.initial_state(o.node_coords(), T))


# --------------------------------------------------------------------------
# shallow water
# --------------------------------------------------------------------------

def _swe_state(rng, cells, flowing=True):
    Cy, Cx = cells[1], cells[0]
    b = 0.3 * rng.random((Cy, Cx))
    h = 1.5 + 0.6 * rng.random((Cy, Cx))
    u = (0.8 * rng.standard_normal((Cy, Cx))) if flowing else 0.0 * h
    v = (0.8 * rng.standard_normal((Cy, Cx))) if flowing else 0.0 * h
    return np.stack([h, h * u, h * v, b])


def test_brute_swe_step_is_well_balanced_and_conservative():
    """The brute-force update itself: a lake at rest (eta constant, no flow)
    over a rough bottom stays exactly at rest; h is conserved."""
    rng = np.random.default_rng(3)
    U = _swe_state(rng, (7, 5), flowing=False)
    U[0] = 2.0 - U[3]
    V = brute.fv_swe_step(U, 0.01, 0.1, 9.81)
    assert np.abs(V[1:3]).max() < 1e-14
    assert np.abs(V[0] + V[3] - 2.0).max() < 1e-14
    U2 = _swe_state(rng, (7, 5))
    W = brute.fv_swe_step(U2, 0.01, 0.1, 9.81)
    assert np.abs(W - U2).max() > 1e-3
    assert abs(W[0].sum() - U2[0].sum()) < 1e-12 * U2[0].size


@pytest.mark.parametrize("cells,seed", [((6, 5), 1), ((4, 7), 2), ((1, 6), 3), ((5, 1), 4)])
def test_swe_order_zero_is_path_conservative_finite_volumes(oracle_mod, cells, seed):
    """N = 0 on random flowing states over a random bottom: the oracle's step
    equals the textbook first-order update (eq. swe_custom_riemann read as the
    surface-dissipating Rusanov flux plus the halved path integral of the
    non-conservative product)."""
    g = 9.81
    rng = np.random.default_rng(seed)
    U = _swe_state(rng, cells)
    o = oracle_mod.Oracle(2, 0, list(cells), [0.0, 0.0], [c * 0.1 for c in cells], "swe", (g,))
    Q = np.moveaxis(U, 0, -1).reshape(-1, 4, 1)
    o.set_state(Q)
    dt = 0.2 * o.h / 6.0
    o.step(0.0, dt)
    ref = brute.fv_swe_step(U, dt, o.h, g)
    ref_Q = np.moveaxis(ref, 0, -1).reshape(-1, 4, 1)
    assert np.abs(ref_Q - Q).max() > 1e-4  # the step moves the state
    np.testing.assert_allclose(o.get_state(), ref_Q, rtol=0, atol=2e-14 * np.abs(U).max())


@pytest.mark.parametrize("order", [2, 3])
def test_swe_gravity_wave_on_a_stream_converges(oracle_mod, order):
    """A gravity wave of amplitude 1e-7 on the stream v = (0.4, -0.25) over a
    flat bottom, k = 2 pi (1, 2): the L2 error against the linear solution
    decays at rate >= N + 1 - 0.3 (the O(eps^2) nonlinear defect is far below
    the discretisation error at these grids)."""
    sc = small("swe", 2, order, (1, 1), (0, 0), (1, 1), (9.81,), "swe_gravity_wave", {"eps": 1e-7},
               cfl=0.45)
    e1 = _error_at(oracle_mod, sc, (6, 6), 0.1)
    e2 = _error_at(oracle_mod, sc, (12, 12), 0.1)
    eoc = math.log2(e1 / e2)
    assert eoc >= order + 1 - 0.3, (e1, e2, eoc)
    # and the error is small against the wave itself (||h'|| ~ 0.7e-7 eps-units)
    assert e2 < 0.05 * 1e-7


def test_swe_gravity_wave_solution_satisfies_linearised_system():
    """The closed form solves the linearised eq. swe (central differences in
    space and time at random points)."""
    g, H, U0 = 9.81, 2.0, (0.4, -0.25)
    rng = np.random.default_rng(0)
    pts = rng.random((16, 3))
    e = 1e-5
    eps = 1e-3

    def state(x, y, t):
        c = [np.array([[x]]), np.array([[y]])]
        return inputs.swe_gravity_wave(c, t, g, depth=H, flow=U0, eps=eps)[0, :, 0]

    for x, y, t in pts:
        q = state(x, y, t)
        dt_ = (state(x, y, t + e) - state(x, y, t - e)) / (2 * e)
        dx_ = (state(x + e, y, t) - state(x - e, y, t)) / (2 * e)
        dy_ = (state(x, y + e, t) - state(x, y - e, t)) / (2 * e)
        hp_t, hp_x, hp_y = dt_[0], dx_[0], dy_[0]
        # perturbation velocities v' = (hu/h - U0)
        def vel(s):
            return np.array([s[1] / s[0] - U0[0], s[2] / s[0] - U0[1]])
        vp_t = (vel(state(x, y, t + e)) - vel(state(x, y, t - e))) / (2 * e)
        vp_x = (vel(state(x + e, y, t)) - vel(state(x - e, y, t))) / (2 * e)
        vp_y = (vel(state(x, y + e, t)) - vel(state(x, y - e, t))) / (2 * e)
        r_h = hp_t + U0[0] * hp_x + U0[1] * hp_y + H * (vp_x[0] + vp_y[1])
        r_v = vp_t + U0[0] * vp_x + U0[1] * vp_y + g * np.array([hp_x, hp_y])
        scale = eps * 30.0
        assert abs(r_h) < 1e-4 * scale and np.abs(r_v).max() < 1e-4 * scale, (r_h, r_v)


# --------------------------------------------------------------------------
# 3-D elastic waves
# --------------------------------------------------------------------------

def _oblique_box(order):
    """P + two S waves along k = 2 pi (1, 1/2, 1/3) on [0,1]x[0,2]x[0,3]."""
    k = np.array([2 * math.pi, math.pi, 2 * math.pi / 3])
    s1 = np.array([math.pi, -2 * math.pi, 0.0])
    pols = [(1.0, k), (0.7, s1), (0.4, np.cross(k, s1))]
    return small("elastic", 3, order, (1, 2, 3), (0, 0, 0), (1, 2, 3), (1.0, 2.0, 1.0),
                 "elastic_plane_waves", {"k": tuple(k), "pols": pols}, cfl=0.5)


def test_elastic_plane_wave_closed_form_matches_paper_matrices():
    """For a wave vector and polarisations in the (x, y) plane the 3-D closed
    form restricted to (sxx, syy, sxy, vx, vy) solves q_t + A q_x + B q_y = 0
    with the matrices printed in the paper (golden file)."""
    rho, lam, mu = 1.3, 2.0, 0.7
    A = paper_matrix("elastic", "A", rho=rho, lam=lam, mu=mu)
    B = paper_matrix("elastic", "B", rho=rho, lam=lam, mu=mu)
    k = np.array([2.0, 1.0, 0.0])
    pols = [(1.0, k), (0.6, np.array([1.0, -2.0, 0.0]))]
    sel = [0, 1, 3, 6, 7]  # sxx, syy, sxy, vx, vy
    e = 1e-5
    rng = np.random.default_rng(1)
    for x, y, t in rng.random((8, 3)):
        def q(x_, y_, t_):
            c = [np.array([[x_]]), np.array([[y_]]), np.array([[0.3]])]
            return inputs.elastic_plane_waves(c, t_, rho, lam, mu, k, pols)[0, :, 0]
        qt = (q(x, y, t + e) - q(x, y, t - e)) / (2 * e)
        qx = (q(x + e, y, t) - q(x - e, y, t)) / (2 * e)
        qy = (q(x, y + e, t) - q(x, y - e, t)) / (2 * e)
        r = qt[sel] + A @ qx[sel] + B @ qy[sel]
        assert np.abs(r).max() < 1e-6 * np.abs(qt).max(), r
        # the out-of-plane shear stresses and velocity stay zero for in-plane data
        assert np.abs(q(x, y, t)[[4, 5, 8]]).max() < 1e-12 * np.abs(q(x, y, t)).max()


def test_elastic_plane_waves_move_every_component():
    sc = _oblique_box(2)
    rng = np.random.default_rng(5)
    coords = [L * rng.random((5, 3)) for L in (1.0, 2.0, 3.0)]
    Q = np.stack([inputs.evaluate(sc, coords, t) for t in (0.0, 0.37, 0.81)])
    amp = np.abs(Q).max(axis=(0, 1, 3))
    assert (amp > 0.05 * amp.max()).all(), amp
    # sigma_yz and sigma_xz are different fields
    assert np.abs(Q[:, :, 4] - Q[:, :, 5]).max() > 0.05 * amp.max()
    assert np.abs(Q[:, :, 4] + Q[:, :, 5]).max() > 0.05 * amp.max()


def test_elastic3d_oblique_plane_waves_converge(oracle_mod):
    """3-D elastic, N = 3, box [0,1]x[0,2]x[0,3] (cells 2x4x6 -> 4x8x12): the L2
    error against the superposed P and S waves decays at rate >= N + 1 - 0.3."""
    sc = _oblique_box(3)
    e1 = _error_at(oracle_mod, sc, (2, 4, 6), 0.1)
    e2 = _error_at(oracle_mod, sc, (4, 8, 12), 0.1)
    eoc = math.log2(e1 / e2)
    assert eoc >= 3.7, (e1, e2, eoc)


def test_elastic3d_benchmark_wave_converges(oracle_mod):
    """The 3-D elastic benchmark state (P and S waves along 2 pi (1,1,1), rho =
    2.7, cp = 6, cs = 3.464) at N = 3 on 3^3 -> 6^3 cells of the unit cube."""
    base = inputs.SCENARIOS["elastic3d_n5_64"]
    sc = small("elastic", 3, 3, (1, 1, 1), (0, 0, 0), (1, 1, 1), base.params, base.ic, base.extra,
               cfl=0.5)
    e1 = _error_at(oracle_mod, sc, (3, 3, 3), 0.02)
    e2 = _error_at(oracle_mod, sc, (6, 6, 6), 0.02)
    eoc = math.log2(e1 / e2)
    assert eoc >= 3.7, (e1, e2, eoc)
