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


def rel_l2(o, A, B):
    """Relative L2 (eq. L2gauss norm) of A - B over B."""
    return o.l2(A, B) / max(o.l2(B), 1e-300)


def gpu_solver(sc, cells=None, prec=None, picard_iters=0):
    from paper_2504_06889_amd.aderdg import Solver
    s = Solver.from_scenario(sc, cells=cells, picard_iters=picard_iters)
    if prec is not None:
        s.set_precisions(*prec)
    return s


def run_both(oracle_mod, sc, cells, nsteps, dt=None, prec=("fp64", "fp64", "fp64"), noise=0.0,
             material=None, source=None, seed=0, emulate=False):
    """Same seeded input through the oracle (FP64 unless emulate) and the GPU path."""
    o = make_oracle(oracle_mod, sc, cells, prec=prec if emulate else ("fp64",) * 3)
    Q0 = sc.initial_state(o.node_coords())
    if noise:
        scale = max(np.abs(Q0).max(), 1.0)
        Q0 = Q0 + noise * scale * np.random.default_rng(seed).standard_normal(Q0.shape)
    o.set_state(Q0)
    if material is not None:
        o.set_material(material)
    if source is not None:
        o.set_source(*source)
    if dt is None:
        dt = o.max_dt(sc.cfl)
    A = o.run(nsteps, dt)
    g = gpu_solver(sc, cells, prec=prec)
    if material is not None:
        g.set_material(material)
    if source is not None:
        g.set_source(*source)
    g.set_state(Q0)
    g.step(dt, nsteps)
    B = g.get_state()
    return o, A, B, dt, g
