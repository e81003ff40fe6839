"""Write the full-length FP64 oracle references of the benchmark workloads.

For each workload the plain FP64 CPU oracle (``oracle/``) runs the whole grid
from the closed-form initial state for the workload's own number of steps, at
the time step of eq. CFL_condition computed from the initial state; the file
``fullsize_<name>.npz`` keeps

  ids      sampled cell ids (the corners of the periodic box, so every
           wrap-around neighbour is involved, plus seeded random cells),
  Q        the oracle's final state at those cells [len(ids), V, S],
  dt, nsteps, cfl, threads, seconds,
  totals   sum over the whole grid of h^d W_i Q_v per variable (eq. L2gauss
           quadrature of each conserved quantity),
  norm     the eq. L2gauss norm of the whole final state, per variable.

Only ``oracle/`` and the input generators (``paper_2504_06889_amd/inputs.py``,
closed-form states, no method arithmetic) are used.  The run is long
(hours for the 64^3 elastic workload on a few cores); ``--ckpt DIR`` saves the
state every ``--every`` steps and resumes from the latest save.

    python tests/golden/make_fullsize.py elastic3d_n5_64 euler3d_n4_48 swe2d_n6_512 --ckpt /tmp/ck
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2504_06889_amd import inputs  # noqa: E402

# sampled cells per workload (the file stays small: V*S doubles per cell)
NSAMPLE = {"elastic3d_n5_64": 32, "euler3d_n4_48": 64, "swe2d_n6_512": 128}


def sample_ids(cells, m, seed):
    """Corners of the box plus m seeded random cells (unique, sorted)."""
    d = len(cells)
    pick = [[(cells[j] - 1) if (corner >> j) & 1 else 0 for j in range(d)] for corner in range(2 ** d)]
    rng = np.random.default_rng(seed)
    while len(pick) < m:
        pick.append([int(rng.integers(0, cells[j])) for j in range(d)])
    ids = []
    for idx in pick:
        c, mult = 0, 1
        for j in range(d):
            c += idx[j] * mult
            mult *= cells[j]
        ids.append(c)
    return np.unique(np.array(ids, dtype=np.int64))


def path(name):
    return os.path.join(HERE, "fullsize_%s.npz" % name)


def run(name, ckpt=None, every=10):
    sc = inputs.SCENARIOS[name]
    o = oracle.Oracle(sc.dim, sc.order, sc.cells, sc.lo, sc.hi, sc.pde, sc.params)
    Q0 = sc.initial_state(o.node_coords())
    o.set_state(Q0)
    dt = o.max_dt(sc.cfl)
    del Q0
    start, seconds = 0, 0.0
    ck = None
    if ckpt:
        os.makedirs(ckpt, exist_ok=True)
        ck = os.path.join(ckpt, name)
        if os.path.exists(ck + ".json"):
            import json
            with open(ck + ".json") as f:
                meta = json.load(f)
            if meta["dt"] == dt:
                o.set_state(np.load(ck + ".npy"))
                start, seconds = meta["step"], meta["seconds"]
                print("%s: resumed at step %d" % (name, start), flush=True)
    for k in range(start, sc.steps):
        t0 = time.time()
        o.step(k * dt, dt)
        seconds += time.time() - t0
        print("%s: step %d/%d (%.1f s)" % (name, k + 1, sc.steps, seconds), flush=True)
        if ck and ((k + 1) % every == 0) and k + 1 < sc.steps:
            import json
            np.save(ck + ".tmp.npy", o.get_state())
            os.replace(ck + ".tmp.npy", ck + ".npy")
            with open(ck + ".json", "w") as f:
                json.dump({"step": k + 1, "dt": dt, "seconds": seconds}, f)
    Q = o.get_state()
    ids = sample_ids(sc.cells, NSAMPLE[name], seed=len(name))
    W = o.weights()
    totals = np.einsum("cvs,s->v", Q, W) * o.h ** o.d
    norm = np.sqrt(np.einsum("cvs,s->v", Q * Q, W) * o.h ** o.d)
    np.savez_compressed(path(name), ids=ids, Q=Q[ids], dt=dt, nsteps=sc.steps, cfl=sc.cfl,
                        threads=oracle.num_threads(), seconds=seconds, totals=totals, norm=norm)
    print("%s: wrote %s (%d cells, %.0f s)" % (name, path(name), ids.size, seconds), flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+")
    ap.add_argument("--ckpt", default=None)
    ap.add_argument("--every", type=int, default=10)
    args = ap.parse_args()
    for nm in args.names:
        run(nm, args.ckpt, args.every)
