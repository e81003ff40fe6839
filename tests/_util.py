"""Shared helpers for the tests (not collected)."""
import json
import os

import numpy as np

from paper_2504_06889_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def paper_matrix(pde, name, **sym):
    """A 2-D flux matrix as printed in the paper (tests/golden/paper_matrices.json)."""
    with open(os.path.join(GOLDEN, "paper_matrices.json")) as f:
        data = json.load(f)
    rows = data[pde][name]
    sym = {("lam" if k == "lambda" else k): v for k, v in sym.items()}
    return np.array([[float(eval(e.replace("lambda", "lam"), {"__builtins__": {}}, sym))
                      for e in r] for r in rows])


def make_oracle(oracle_mod, sc, cells=None, prec=("fp64", "fp64", "fp64"), picard_iters=0):
    cells = sc.cells if cells is None else cells
    return oracle_mod.Oracle(sc.dim, sc.order, cells, sc.lo, sc.hi, sc.pde, sc.params,
                             picard_iters=picard_iters, prec=prec)


def scenario(name, **changes):
    sc = inputs.SCENARIOS[name]
    sc = inputs.Scenario(**{**sc.__dict__, **changes})
    return sc


def small(pde, dim, order, cells, lo, hi, params, ic, extra=None, cfl=0.5):
    return inputs.Scenario("test", pde, dim, order, tuple(cells), tuple(lo), tuple(hi),
                           tuple(params), 1, cfl, ic, dict(extra or {}))


def run_oracle(o, sc, nsteps, dt, t0=0.0, Q0=None):
    if Q0 is None:
        Q0 = sc.initial_state(o.node_coords(), t0)
    o.set_state(Q0)
    return o.run(nsteps, dt, t0)
