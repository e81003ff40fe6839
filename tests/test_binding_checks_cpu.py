"""The binding refuses a wrong tensor before its pointer reaches the library
(no GPU needed: the dtype, contiguity and size checks come first)."""
import pytest
import torch

from paper_2504_06889_amd.aderdg import Solver, check_tensor


def _fake_solver():
    # a Solver shell with the geometry fields only (no library handle)
    s = object.__new__(Solver)
    s._h = None
    s.ncell, s.V, s.S, s.nrec, s.device = 8, 4, 27, 3, 0
    return s


def test_check_tensor_order_of_checks():
    with pytest.raises(ValueError, match="float64"):
        check_tensor(torch.zeros(4, dtype=torch.float32), "x", 4)
    with pytest.raises(ValueError, match="contiguous"):
        check_tensor(torch.zeros(4, 2, dtype=torch.float64).t(), "x", 8)
    with pytest.raises(ValueError, match="elements"):
        check_tensor(torch.zeros(5, dtype=torch.float64), "x", 4)
    with pytest.raises(ValueError, match="device"):
        check_tensor(torch.zeros(4, dtype=torch.float64), "x", 4)
    with pytest.raises(ValueError, match="torch tensor"):
        check_tensor([0.0] * 4, "x", 4)


@pytest.mark.parametrize("which", ["Qn", "lam", "grad"])
@pytest.mark.parametrize("bad", ["dtype", "size"])
def test_step_adjoint_refuses_bad_tensors(which, bad):
    s = _fake_solver()
    n = s.ncell * s.V * s.S
    t = {"Qn": torch.zeros(n, dtype=torch.float64), "lam": torch.zeros(n, dtype=torch.float64),
         "grad": torch.zeros(s.ncell, dtype=torch.float64)}
    x = t[which]
    t[which] = x.to(torch.float32) if bad == "dtype" else torch.zeros(x.numel() - 1, dtype=torch.float64)
    with pytest.raises(ValueError, match=which):
        s.step_adjoint(0.1, 0.0, t["Qn"], t["lam"], t["grad"])


def test_receivers_adjoint_and_material_refuse_bad_tensors():
    s = _fake_solver()
    n = s.ncell * s.V * s.S
    with pytest.raises(ValueError, match="weight"):
        s.receivers_adjoint(torch.zeros(s.nrec, dtype=torch.float32), torch.zeros(n, dtype=torch.float64))
    with pytest.raises(ValueError, match="lam"):
        s.receivers_adjoint(torch.zeros(s.nrec, dtype=torch.float64), torch.zeros(n + 1, dtype=torch.float64))
    with pytest.raises(ValueError, match="c must hold"):
        s.set_material([1.0] * (s.ncell - 1))
