"""GPU adjoint (through the C ABI and the autograd Function) against the CPU
oracle's reverse-mode adjoint, the dot-product identity and central finite
differences."""
import numpy as np
import pytest

from oracle import misfit as omisfit
from paper_2504_06889_amd import inputs

pytestmark = pytest.mark.gpu


def _setup(oracle_mod, dim, order, cells, L=1.0, source=True, seed=0):
    import torch
    from paper_2504_06889_amd.aderdg import Solver
    h = L / max(cells)
    hi = tuple(c * h for c in cells)
    o = oracle_mod.Oracle(dim, order, cells, (0.0,) * dim, hi, "acoustic", (1.0, 2.25))
    g = Solver(dim, order, cells, (0.0,) * dim, hi, "acoustic", (1.0, 2.25))
    c = inputs.lognormal_speed(o.ncell, mean=1.5, sigma=0.2, seed=seed)
    o.set_material(c)
    g.set_material(c)
    xs = [0.5 * L + 0.1 * h, 0.5 * hi[1] - 0.2 * h] + ([0.5 * hi[2] + 0.05 * h] if dim == 3 else [])
    if source:
        o.set_source(xs, 5.0, 0.2, 1.0)
        g.set_source(xs, 5.0, 0.2, 1.0)
    dt = 0.5 * h / (dim * (2 * order + 1) * c.max())
    return o, g, c, xs, dt, torch


@pytest.mark.parametrize("dim,order,cells", [(3, 2, (3, 4, 2)), (3, 5, (2, 3, 2)), (2, 3, (5, 4)),
                                             (3, 1, (4, 3, 5)), (2, 2, (7, 3))])
def test_adjoint_step_matches_oracle(oracle_mod, dim, order, cells):
    o, g, c, xs, dt, torch = _setup(oracle_mod, dim, order, cells, seed=dim + order)
    print("case", dim, order, cells, flush=True)
    rng = np.random.default_rng(order)
    Qn = rng.standard_normal(o.shape)
    lam = rng.standard_normal(o.shape)
    t = 0.13
    mu_o, g_o = o.adjoint_step(Qn, t, dt, lam, np.zeros(o.ncell))
    Qd = torch.from_numpy(Qn).cuda()
    ld = torch.from_numpy(lam).cuda()
    gd = torch.zeros(o.ncell, dtype=torch.float64, device="cuda")
    g.step_adjoint(dt, t, Qd, ld, gd)
    mu_g, g_g = ld.cpu().numpy(), gd.cpu().numpy()
    assert np.linalg.norm(mu_g - mu_o) <= 1e-10 * np.linalg.norm(mu_o)
    assert np.linalg.norm(g_g - g_o) <= 1e-10 * np.linalg.norm(g_o), (np.linalg.norm(g_g - g_o), np.linalg.norm(g_o))
    # the incoming state is not modified
    np.testing.assert_array_equal(Qd.cpu().numpy(), Qn)


def test_adjoint_step_with_stored_faces_is_identical(oracle_mod):
    """The forward face data copied right after a step (aderdg_copy_faces) give the
    same adjoint step, bit for bit, as recomputing them from the state."""
    o, g, c, xs, dt, torch = _setup(oracle_mod, 3, 5, (3, 2, 4), seed=3)
    rng = np.random.default_rng(5)
    Qn = torch.from_numpy(rng.standard_normal(o.shape)).cuda()
    lam = rng.standard_normal(o.shape)
    t = 0.07
    g.set_state(Qn)
    g.time = t
    g.step(dt, 1)
    faces = g.copy_faces(torch.empty(g.face_bytes(), dtype=torch.uint8, device="cuda"))
    l1, l2 = torch.from_numpy(lam).cuda(), torch.from_numpy(lam).cuda()
    g1 = torch.zeros(o.ncell, dtype=torch.float64, device="cuda")
    g2 = torch.zeros(o.ncell, dtype=torch.float64, device="cuda")
    g.step_adjoint(dt, t, Qn, l1, g1)
    g.step_adjoint(dt, t, Qn, l2, g2, fwd_faces=faces)
    assert torch.equal(l1, l2) and torch.equal(g1, g2)


def test_adjoint_step_dot_product_on_gpu(oracle_mod):
    o, g, c, xs, dt, torch = _setup(oracle_mod, 3, 5, (3, 2, 2), source=False)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(o.shape)
    w = rng.standard_normal(o.shape)
    g.set_state(v)
    g.step(dt, 1)
    Jv = g.get_state()
    wd = torch.from_numpy(w).cuda()
    g.step_adjoint(dt, 0.0, torch.from_numpy(v).cuda(), wd, torch.zeros(o.ncell, dtype=torch.float64,
                                                                          device="cuda"))
    lhs, rhs = float(np.sum(w * Jv)), float(np.sum(wd.cpu().numpy() * v))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("checkpoint", [1, 7, 30])
def test_misfit_gradient_matches_oracle_and_differences(oracle_mod, checkpoint):
    from paper_2504_06889_amd import adjoint as adj
    o, g, c, xs, dt, torch = _setup(oracle_mod, 3, 2, (4, 4, 4), L=2.0, seed=5)
    rec = inputs.receivers_near(xs, o.h, nrec=8, half_cells=1.5, seed=1)
    g.set_receivers(rec)
    nsteps = 30
    Q0 = np.zeros(o.shape)
    Q0d = torch.from_numpy(Q0).cuda()
    # synthetic data: the same forward with a homogeneous c = 1.5
    data = adj.record(g, torch.full((o.ncell,), 1.5, dtype=torch.float64, device="cuda"), Q0d, dt, nsteps)
    cd = torch.from_numpy(c).cuda().requires_grad_(True)
    J = adj.misfit(cd, g, Q0d, dt, nsteps, data, checkpoint)
    J.backward()
    grad = cd.grad.cpu().numpy()
    # oracle: same misfit, reverse-mode gradient
    Jo, go, _ = omisfit.gradient(o, Q0, c, dt, nsteps, rec, data.cpu().numpy())
    assert abs(float(J) - Jo) <= 1e-10 * Jo
    assert np.linalg.norm(grad - go) <= 1e-10 * np.linalg.norm(go)
    # central differences of the GPU misfit along a random direction
    dc = np.random.default_rng(2).standard_normal(o.ncell)
    eps = 1e-6 * np.linalg.norm(c) / np.linalg.norm(dc)

    def Jof(cc):
        with torch.no_grad():
            return float(adj.misfit(torch.from_numpy(cc).cuda(), g, Q0d, dt, nsteps, data, checkpoint))
    fd = (Jof(c + eps * dc) - Jof(c - eps * dc)) / (2 * eps)
    assert abs(fd - grad @ dc) <= 1e-6 * abs(fd), (fd, grad @ dc)


def test_receiver_adjoint_scatter_is_deterministic(oracle_mod):
    """Many receivers in few cells: the scatter sums each cell's receivers in a
    fixed order, so two calls give bitwise-equal results, equal to the sum of the
    receivers' nodal weights (oracle point weights) to rounding."""
    import torch
    from paper_2504_06889_amd.aderdg import Solver
    dim, order, cells = 3, 5, (3, 3, 2)
    hi = tuple(c / 3.0 for c in cells)
    o = oracle_mod.Oracle(dim, order, cells, (0.0,) * dim, hi, "acoustic", (1.0, 2.25))
    g = Solver(dim, order, cells, (0.0,) * dim, hi, "acoustic", (1.0, 2.25))
    rng = np.random.default_rng(7)
    # 200 receivers in the 2 x 2 x 1 block of cells at the origin
    pts = rng.uniform(0.0, 1.0, size=(200, dim)) * np.array([2 / 3.0, 2 / 3.0, 1 / 3.0])
    g.set_receivers(pts)
    w = rng.standard_normal(200)
    ref = np.zeros(o.shape)
    for r in range(200):
        cell, phi = o.point_weights(pts[r])
        ref[cell, 0] += w[r] * phi
    wd = torch.from_numpy(w).cuda()
    outs = []
    for _ in range(2):
        lam = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
        g.receivers_adjoint(wd, lam)
        outs.append(lam.cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])
    assert np.abs(outs[0] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_misfit_gradient_order5_across_checkpoint_segments(oracle_mod):
    """Order 5 (the adjoint configuration's order), 3^3 cells, 40 steps, checkpoint
    every 20 (the sweep recomputes two segments): gradient against the oracle's
    reverse mode (1e-10) and central differences (1e-6); two backward sweeps give
    bitwise-equal gradients (receivers sharing cells)."""
    from paper_2504_06889_amd import adjoint as adj
    o, g, c, xs, dt, torch = _setup(oracle_mod, 3, 5, (3, 3, 3), L=1.5, seed=9)
    rec = inputs.receivers_near(xs, o.h, nrec=12, half_cells=1.0, seed=3)
    g.set_receivers(rec)
    nsteps, K = 40, 20
    Q0 = np.zeros(o.shape)
    Q0d = torch.from_numpy(Q0).cuda()
    data = adj.record(g, torch.full((o.ncell,), 1.5, dtype=torch.float64, device="cuda"), Q0d, dt, nsteps)
    grads = []
    for _ in range(2):
        cd = torch.from_numpy(c).cuda().requires_grad_(True)
        J = adj.misfit(cd, g, Q0d, dt, nsteps, data, K)
        J.backward()
        grads.append(cd.grad.detach().clone())
    assert torch.equal(grads[0], grads[1])
    grad = grads[0].cpu().numpy()
    Jo, go, _ = omisfit.gradient(o, Q0, c, dt, nsteps, rec, data.cpu().numpy())
    assert abs(float(J.detach()) - Jo) <= 1e-10 * Jo
    assert np.linalg.norm(grad - go) <= 1e-10 * np.linalg.norm(go), np.linalg.norm(grad - go) / np.linalg.norm(go)
    dc = np.random.default_rng(4).standard_normal(o.ncell)
    eps = 1e-6 * np.linalg.norm(c) / np.linalg.norm(dc)

    def Jof(cc):
        with torch.no_grad():
            return float(adj.misfit(torch.from_numpy(cc).cuda(), g, Q0d, dt, nsteps, data, K))
    fd = (Jof(c + eps * dc) - Jof(c - eps * dc)) / (2 * eps)
    assert abs(fd - grad @ dc) <= 1e-6 * abs(fd), (fd, grad @ dc)
