"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function include/aderdg.h declares, and its host-built basis agrees with the
oracle's."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aderdg.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(aderdg_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2504_06889_amd import aderdg
    if not os.path.exists(aderdg.LIB_PATH):
        pytest.skip("libaderdg.so not built")
    return aderdg.LIB_PATH


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (aderdg_[a-z_]+)\b", out))
    declared = _declared()
    assert declared, "no declarations found"
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    from paper_2504_06889_amd import aderdg
    assert sorted(aderdg.EXPORTS) == declared
    lib = aderdg.lib()
    for f in declared:
        assert hasattr(lib, f)


@pytest.mark.parametrize("n", range(1, 9))
def test_library_nodes_match_oracle(libpath, oracle_mod, n):
    from paper_2504_06889_amd import aderdg
    xi, w = aderdg.nodes(n)
    b = oracle_mod.basis(n)
    np.testing.assert_allclose(xi, b["xi"], atol=2e-15, rtol=0)
    np.testing.assert_allclose(w, b["w"], atol=2e-15, rtol=0)


def test_library_rejects_bad_node_count(libpath):
    from paper_2504_06889_amd import aderdg
    with pytest.raises(aderdg.AderdgError):
        aderdg.nodes(0)
    with pytest.raises(aderdg.AderdgError):
        aderdg.nodes(9)


def test_binding_refuses_to_run_without_gpu(libpath):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2504_06889_amd.aderdg import Solver
    with pytest.raises(RuntimeError):
        Solver(2, 3, (4, 4), (0, 0), (1, 1), "acoustic", (1.0, 1.0))


@pytest.mark.parametrize("cells", [(2048, 1024, 1024), (4, 0, 4)])
def test_create_validates_grid_before_touching_the_device(libpath, cells):
    """Grids of 2^31 or more cells (the kernels index cells in 32 bits) and empty
    dimensions are rejected with INVALID before any device call."""
    import ctypes
    from paper_2504_06889_amd import aderdg
    c = aderdg._Config()
    c.dim, c.order, c.pde = 3, 1, aderdg.PDE["elastic"]
    for k in range(3):
        c.cells[k], c.lo[k], c.hi[k] = cells[k], 0.0, float(max(cells[k], 1))
    for k, v in enumerate((1.0, 2.0, 1.0)):
        c.params[k] = v
    h = ctypes.c_void_p()
    rc = aderdg.lib().aderdg_create(ctypes.byref(c), None, ctypes.byref(h))
    assert rc == -1 and not h.value
    msg = aderdg.lib().aderdg_last_error(None).decode()
    assert ("2^31" in msg) if cells[1] else ("positive" in msg)
