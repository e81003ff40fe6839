"""The adjoint entry point that allocates nothing (aderdg_step_adjoint_faces_noalloc,
the library's static scratch array) against aderdg_step_adjoint_faces, bit for bit:
two calls in a row, the second on a smaller grid, in FP64 and in the mixed-precision
adjoint; grids beyond the array are refused."""
import numpy as np
import pytest

from paper_2504_06889_amd import inputs

pytestmark = pytest.mark.gpu


def _case(dim, order, cells, prec, seed):
    import torch
    from paper_2504_06889_amd.aderdg import Solver
    h = 1.0 / max(cells)
    hi = tuple(c * h for c in cells)
    g = Solver(dim, order, cells, (0.0,) * dim, hi, "acoustic", (1.0, 2.25))
    g.set_precisions(prec, prec, "fp64")
    ncell = int(np.prod(cells))
    c = inputs.lognormal_speed(ncell, mean=1.5, sigma=0.2, seed=seed)
    g.set_material(c)
    xs = [0.5 * hi[0] + 0.1 * h, 0.5 * hi[1] - 0.2 * h] + ([0.5 * hi[2] + 0.05 * h] if dim == 3 else [])
    g.set_source(xs, 5.0, 0.2, 1.0)
    dt = 0.5 * h / (dim * (2 * order + 1) * c.max())
    rng = np.random.default_rng(seed)
    Qn = torch.from_numpy(rng.standard_normal(g.shape)).cuda()
    lam = torch.from_numpy(rng.standard_normal(g.shape)).cuda()
    t = 0.11
    g.set_state(Qn)
    g.time = t
    g.step(dt, 1)
    faces = g.copy_faces(torch.empty(g.face_bytes(), dtype=torch.uint8, device="cuda"))
    return g, Qn, lam, faces, dt, t, torch


@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_noalloc_adjoint_matches_allocating_entry_point(prec):
    # the second call runs on a smaller grid: the array keeps the first call's
    # contents beyond the second one's range, which must not leak into it
    for dim, order, cells, seed in [(3, 5, (4, 5, 3), 1), (3, 5, (2, 3, 2), 2)]:
        print("case", prec, dim, order, cells, flush=True)
        g, Qn, lam, faces, dt, t, torch = _case(dim, order, cells, prec, seed)
        lam_a, grad_a = lam.clone(), torch.zeros(g.ncell, dtype=torch.float64, device="cuda")
        lam_b, grad_b = lam.clone(), torch.zeros(g.ncell, dtype=torch.float64, device="cuda")
        g.step_adjoint(dt, t, Qn, lam_a, grad_a, fwd_faces=faces)
        g.step_adjoint_noalloc(dt, t, Qn, lam_b, grad_b, faces)
        torch.cuda.synchronize()
        assert torch.isfinite(lam_b).all()
        assert torch.equal(lam_a, lam_b)
        assert torch.equal(grad_a, grad_b)
        assert float(lam_b.abs().max()) > 0


def test_noalloc_adjoint_refuses_grids_beyond_the_array():
    from paper_2504_06889_amd.aderdg import AderdgError
    # 3-D order 5 acoustics: 6912 bytes of face restrictions per cell; 22^3 cells
    # need 73.6 MB > 64 MiB
    g, Qn, lam, faces, dt, t, torch = _case(3, 5, (22, 22, 22), "fp64", 3)
    grad = torch.zeros(g.ncell, dtype=torch.float64, device="cuda")
    before = lam.clone()
    with pytest.raises(AderdgError) as e:
        g.step_adjoint_noalloc(dt, t, Qn, lam, grad, faces)
    assert e.value.code == -1 and "scratch" in str(e.value)
    assert torch.equal(lam, before)
