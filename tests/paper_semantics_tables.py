"""The paper's 2-D scenarios under the oracle's emulation of the paper's own
precision semantics (each kernel computes, accumulates and stores in its type;
Sec. 4.1, the runs of Sec. 7), on a reduced grid, for comparison of trends with
the paper's tables and with the GPU path's runs of the same settings; with
--semantics build the same settings run under the emulation of the library's own
rounding points instead, on the same grid.

Not collected by pytest (a script of the test infrastructure): it runs the CPU
oracle only and prints one JSON line per scenario.  Settings are (predictor,
Picard, corrector, storage) types; "predictor" is the paper's fused predictor
kernel (Picard loop, time averages, face projection, volume integral), its Picard
loop takes the Picard type, "corrector" the Riemann solve and surface integral.

    python tests/paper_semantics_tables.py --cells 9 --threads 4
    python tests/paper_semantics_tables.py --cells 9 --threads 4 --semantics build
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2504_06889_amd import inputs  # noqa: E402


def settings():
    """(label, predictor, Picard, corrector, storage)."""
    out = [("fp64", "fp64", "fp64", "fp64", "fp64"), ("all+storage=fp32", "fp32", "fp32", "fp32", "fp32")]
    for p in ("fp32", "bf16", "fp16"):
        out.append(("storage64:predictor=%s" % p, p, p, "fp64", "fp64"))
        out.append(("storage64:corrector=%s" % p, "fp64", "fp64", p, "fp64"))
    for p in ("bf16", "fp16"):
        out.append(("storage32:predictor=%s" % p, p, p, "fp32", "fp32"))
    for k in ("Picard", "predictor", "corrector", "all"):
        pr = "fp64" if k in ("predictor", "all") else "fp32"
        pq = "fp64" if k in ("Picard", "predictor", "all") else "fp32"
        co = "fp64" if k in ("corrector", "all") else "fp32"
        out.append(("base32:%s=fp64" % k, pr, pq, co, "fp32"))
    return out


def make(sc, pr, pq, co, st, semantics):
    """The oracle in one setting.  Under the paper's semantics the Picard loop has a
    type of its own; under the library's (rounding points of the GPU kernels) the
    Picard loop is the PREDICTOR kernel and the rest of the paper's predictor
    kernel (time averages, projection, volume integral) the VOLUME kernel."""
    if semantics == "paper":
        return oracle.Oracle(sc.dim, sc.order, sc.cells, sc.lo, sc.hi, sc.pde, sc.params, prec=(pr, "fp64", co),
                             storage=st, semantics="paper", prec_picard=pq)
    return oracle.Oracle(sc.dim, sc.order, sc.cells, sc.lo, sc.hi, sc.pde, sc.params, prec=(pq, pr, co),
                         storage=st)


def run(name, cells, semantics="paper"):
    sc = inputs.PAPER_SUITE[name].with_cells((cells, cells))
    res = {}
    ref = None
    for label, pr, pq, co, st in settings():
        o = make(sc, pr, pq, co, st, semantics)
        X = o.node_coords()
        Q0 = sc.initial_state(X)
        o.set_state(Q0)
        t_end = sc.extra["t_end"]
        if ref is None:
            nsteps = int(math.ceil(t_end / o.max_dt(sc.cfl)))
            dt = t_end / nsteps
            exact = sc.initial_state(X, t_end)
        t0 = time.time()
        ok = True
        for k in range(nsteps):
            o.step(k * dt, dt)
            if k % 200 == 199 and not np.all(np.isfinite(o.get_state())):
                ok = False
                break
        Q = o.get_state()
        r = {"seconds": time.time() - t0}
        if not ok or not np.all(np.isfinite(Q)):
            r["error"] = "non-finite"
        else:
            if ref is None:
                ref = Q
            r["l2_vs_exact"] = o.l2(Q, exact)
            r["l2_rel_vs_fp64"] = o.l2(Q, ref) / o.l2(ref)
            if sc.pde == "swe":
                r["max_abs_momentum"] = float(np.abs(Q[:, 1:3]).max())
        res[label] = r
        print(name, label, {k: ("%.3g" % v if isinstance(v, float) else v) for k, v in r.items()},
              file=sys.stderr, flush=True)
    return {"cells": [cells, cells], "order": sc.order, "t_end": sc.extra["t_end"], "steps": nsteps, "dt": dt,
            "semantics": semantics, "runs": res}


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells", type=int, default=9)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--semantics", choices=["paper", "build"], default="paper")
    ap.add_argument("names", nargs="*")
    args = ap.parse_args()
    if args.threads:
        oracle.set_num_threads(args.threads)
    for nm in args.names or list(inputs.PAPER_SUITE):
        print(json.dumps({nm: run(nm, args.cells, args.semantics)}), flush=True)
