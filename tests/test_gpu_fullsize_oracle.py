"""The benchmark workloads over their full length on the whole grid, in the launch
configuration the benchmark times (one aderdg_step call: fused corrector + predictor
launches), against the full-length FP64 oracle references in tests/golden (written by
tests/golden/make_fullsize.py with the oracle only) at the sampled cells: FP64 to 1e-10
(relative L2 over the sampled cells, and element-wise against each variable's largest
value), the lower-format predictor and volume contractions to the stated tolerances."""
import os

import numpy as np
import pytest

from _util import GOLDEN, gpu_solver
from paper_2504_06889_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-6, "fp16": 1e-3, "bf16": 1e-2}
CASES = [("elastic3d_n5_64", "fp64"), ("elastic3d_n5_64", "fp16"), ("elastic3d_n5_64", "bf16"),
         ("elastic3d_n5_64", "fp32"), ("euler3d_n4_48", "fp64"), ("euler3d_n4_48", "fp16"),
         ("swe2d_n6_512", "fp64"), ("swe2d_n6_512", "fp32")]


def _golden(name):
    path = os.path.join(GOLDEN, "fullsize_%s.npz" % name)
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


@pytest.mark.parametrize("name,p", CASES)
def test_full_length_run_matches_oracle_reference(name, p):
    ref = _golden(name)
    if ref is None:
        pytest.skip("no full-length oracle reference for %s" % name)
    sc = inputs.SCENARIOS[name]
    print("case", name, p, int(ref["nsteps"]), "steps", flush=True)
    g = gpu_solver(sc, prec=("fp64",) * 3 if p == "fp64" else (p, p, "fp64"))
    import torch
    Q0 = torch.from_numpy(sc.initial_state(g.node_coords())).cuda()
    g.set_state(Q0)
    dt = float(ref["dt"])
    assert abs(g.max_dt(sc.cfl) - dt) <= 1e-14 * dt
    g.step(dt, int(ref["nsteps"]))
    ids = torch.from_numpy(ref["ids"]).cuda()
    st = g.get_state(out=torch.empty(g.shape, dtype=torch.float64, device="cuda"))
    B = st.index_select(0, ids).cpu().numpy()
    A = ref["Q"]
    W = g.weights()[None, None, :]
    rel = float(np.sqrt(((B - A) ** 2 * W).sum() / (A ** 2 * W).sum()))
    scale = np.abs(A).max(axis=(0, 2))
    scale = np.maximum(scale, 1e-3 * scale.max())
    elem = float((np.abs(B - A).max(axis=(0, 2)) / scale).max())
    # whole-grid totals (conservation) against the oracle's
    Wf = torch.from_numpy(g.weights()).cuda()
    totals = (st * Wf[None, None, :]).sum(dim=(0, 2)).cpu().numpy() * g.h ** g.d
    tot_err = np.abs(totals - ref["totals"]).max() / np.abs(ref["norm"]).max()
    print("%s %s: sampled rel L2 %.3e, element-wise %.3e, totals %.3e" % (name, p, rel, elem, tot_err),
          flush=True)
    assert np.all(np.isfinite(B))
    assert rel <= TOL[p], rel
    if p == "fp64":
        assert elem <= 1e-10, elem
        assert tot_err <= 1e-12, tot_err
