"""aderdg_copy_faces through the C ABI: the layout and size of the copied face
data, with the q halves alone where the predictor writes no f halves (a linear
PDE with FP64 faces), and device and host copies alike."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DIM, ORDER, CELLS = 2, 3, (5, 4)


def _cellwise_constant(pde, ncell, V, S, rng):
    """A state constant inside each cell: the predictor is cell-local, so its time
    average is that constant and every face value of a cell equals it (Alg. 1)."""
    if pde == "euler":
        rho = 1.0 + 0.2 * rng.random(ncell)
        u = 0.1 * rng.standard_normal((ncell, DIM))
        E = 1.0 / 0.4 + 0.5 * rho * (u ** 2).sum(1)
        val = np.column_stack([rho, rho[:, None] * u, E])
    else:
        val = rng.standard_normal((ncell, V))
    return np.repeat(val[:, :, None], S, axis=2), val


@pytest.mark.parametrize("pde,params,flux,q_only", [("acoustic", (1.0, 2.25), "fp64", True),
                                                    ("acoustic", (1.0, 2.25), "fp32", False),
                                                    ("euler", (1.4,), "fp64", False)])
def test_copy_faces_layout(pde, params, flux, q_only):
    import torch
    from paper_2504_06889_amd.aderdg import Solver, lib
    print("case", pde, flux, flush=True)
    h = 1.0 / max(CELLS)
    g = Solver(DIM, ORDER, CELLS, (0.0,) * DIM, tuple(c * h for c in CELLS), pde, params)
    g.set_precisions("fp64", "fp64", flux)
    V, F, S, ncell = g.V, g.F, g.S, g.ncell
    Q, val = _cellwise_constant(pde, ncell, V, S, np.random.default_rng(7))
    g.set_state(Q)
    g.step(1e-3 * h, 1)
    esize = 8 if flux == "fp64" else 4
    halves = 1 if q_only else 2
    assert g.face_bytes() == ncell * DIM * 2 * halves * V * F * esize
    dev = g.copy_faces(torch.zeros(g.face_bytes(), dtype=torch.uint8, device="cuda")).cpu().numpy()
    host = np.zeros(g.face_bytes(), dtype=np.uint8)
    rc = lib().aderdg_copy_faces(g._h, ctypes.c_void_p(host.ctypes.data), 0)
    assert rc == 0
    np.testing.assert_array_equal(dev, host)
    faces = dev.view(np.float64 if flux == "fp64" else np.float32).reshape(ncell, DIM, 2, halves, V, F)
    expect = np.broadcast_to(val[:, None, None, :, None], (ncell, DIM, 2, V, F))
    tol = 1e-12 if flux == "fp64" else 2e-6
    np.testing.assert_allclose(faces[:, :, :, 0], expect, rtol=tol, atol=tol * np.abs(val).max())
