"""Throughput of the ADER-DG time step on one MI355X.

Workload: 3-D linear elastic waves (9 variables), order N = 5 (6 Gauss-Legendre
nodes per dimension), 64^3 periodic cells on the unit cube, rho = 2.7,
cp = 6.0, cs = 3.464, planar P + S wave; C_CFL = 0.5 in
dt = C h / (d (2N+1) lambda_max).  One step = predictor (Picard iteration),
face projection, volume integral, Rusanov flux and corrector over all cells.

The same K steps are timed for the all-FP64 path and for the predictor and
volume contractions in FP32, BF16 and FP16 on the matrix cores (FP32
accumulate; Picard time operator, time averages, flux/corrector and state in
FP64).  `value` is the FP16 variant's cell-DOF updates/s (DOF = cells * n^3 * 9
per step); every variant's throughput, speed-up over FP64 and L2 error
(eq. L2gauss norm, relative) against the FP64 GPU run and the exact solution
are in `runs`.  Inputs are resident in HBM before the timed region.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32_valu": 157.3e12, "mfma_fp32": 157.3e12, "mfma_bf16": 2.5e15,
        "mfma_fp16": 2.5e15, "hbm": 8.0e12}
TOL = {"fp64": 1e-10, "fp32": 1e-6, "fp16": 1e-3, "bf16": 1e-2}
HEADLINE = "fp16"


def flux_flops(pde, d):
    """Flops of one pointwise flux F_j (one direction, one node)."""
    return {"acoustic": 2, "elastic": 8 if d == 3 else 5, "euler": 3 * d + 7, "swe": 3}[pde]


def predictor_flops(pde, d, N, V, I):
    """Algorithmic flops per cell of one predictor launch (sum-factorised, no
    padding): returns (contraction flops that go to the matrix cores in the
    mixed path, FP64 vector flops, pointwise-flux flops)."""
    n = N + 1
    S = n ** d
    ST = n * S
    F = S // n
    deriv = I * d * 2 * n * ST * V            # D along x, y, z at every time slice
    volume = d * 2 * n * S * V                # Kxi along x, y, z
    time_op = I * 2 * n * ST * V              # q_a <- Q - dt sum_b Atau[a][b] R_b
    adds = I * ST * V * ((d - 1) + 1 + 2)     # sum over directions, 1/h scale, final update
    flux = I * ST * d * flux_flops(pde, d)
    avg = 2 * ST * V + n * S * d * flux_flops(pde, d) + 2 * ST * d * V
    faces = 2 * 2 * d * V * F * 2 * n
    return deriv + volume, time_op + adds + avg + faces, flux


def corrector_flops(d, N, V):
    """Flops per cell of the corrector: Rusanov flux at the d*F nodes of each of the
    2d faces (computed from both sides) and the lift into the S*V state values."""
    n = N + 1
    S = n ** d
    F = S // n
    return 2 * d * F * (6 * V + 20) + 4 * d * V * S


def fused_bytes(d, N, V, face_bytes, q_only):
    """HBM bytes per cell of one fused launch (corrector of the previous step +
    predictor): Q* read and written (FP64), the previous face data of the cell and of
    its neighbours read, the new face data written.  For a linear PDE with FP64 faces
    only the projected q is stored."""
    n = N + 1
    S = n ** d
    F = S // n
    faces = 2 * d * V * F * face_bytes * (1 if q_only else 2)
    return 2 * S * V * 8 + 2 * faces + faces


# Sources that determine the machine code of k_predictor for this workload.
KERNEL_SOURCES = ("paper_2504_06889_amd/csrc/common.h", "paper_2504_06889_amd/csrc/kernels.h",
                  "paper_2504_06889_amd/csrc/registry.h",
                  "paper_2504_06889_amd/csrc/inst_elastic3.hip", "paper_2504_06889_amd/build.py")
TRAFFIC_FILE = "profiles/k_predictor_elastic3d_n5_64_hbm_traffic.md"


def kernel_source_hash():
    """SHA-256 of the kernel sources with comments and blank lines removed (an edit
    of a comment does not change the kernel)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0] if not f.endswith(".py") else line.split("#", 1)[0]
                code = code.strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic():
    """Per-launch HBM bytes of k_predictor from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (scaled by a plain copy's counter readings), or {} when the
    kernel sources have changed since the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return {}
    out, ok = {}, False
    with open(path) as fh:
        for line in fh:
            t = line.strip()
            if t.startswith("kernel-source-sha256:"):
                ok = t.split(":", 1)[1].strip() == kernel_source_hash()
            elif t.startswith("traffic-bytes-per-launch"):
                key, val = t[len("traffic-bytes-per-launch"):].split(":")
                out[key.strip()] = int(val)
    return out if ok else {}


def l2(W, h, d, A, B=None):
    import torch
    diff = A if B is None else A - B
    return float(torch.sqrt((diff * diff * W[None, None, :]).sum() * h ** d))


def cpu_baseline(sc, seconds=12.0, cells=8):
    """The FP64 oracle on a periodic cells^3 sub-grid of the same problem (same
    order, cell size and per-cell work), timed on the host cores."""
    import oracle
    h = (sc.hi[0] - sc.lo[0]) / sc.cells[0]
    o = oracle.Oracle(sc.dim, sc.order, (cells,) * sc.dim, sc.lo, tuple(sc.lo[j] + cells * h for j in range(sc.dim)),
                      sc.pde, sc.params)
    o.set_state(sc.initial_state(o.node_coords()))
    dt = o.max_dt(sc.cfl)
    o.step(0.0, dt)  # warm-up
    steps, t0 = 0, time.perf_counter()
    while True:
        o.step(steps * dt, dt)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 2000:
            break
    dof = o.ncell * o.S * o.V
    return {"value": dof * steps / el, "unit": "cell-DOF updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d FP64 oracle steps of the same problem on a periodic %d^3-cell sub-grid "
                      "(%d cells, same order and cell size), %.1f s" % (steps, cells, o.ncell, el)}


def adjoint_bench(steps=None, checkpoint=None, fd=True, mixed=("fp16", "bf16")):
    """Receiver-misfit gradient on the adjoint configuration: 3-D acoustics N=5,
    64^3 cells on [0,20]^3, log-normal per-cell sound speed (mean 1.5, sigma 0.2,
    seed 0), Ricker source f0=5 at the centre of cell (32,32,32), 64 receivers,
    200 steps, checkpoint every 20.  Times the forward misfit and the backward
    (adjoint) sweep in FP64 and checks the gradient against central differences;
    then the same with the predictor and volume contractions of the forward and
    of the adjoint in each format of `mixed`, against the FP64 gradient."""
    import torch
    from paper_2504_06889_amd import adjoint as adj
    from paper_2504_06889_amd import inputs
    from paper_2504_06889_amd.aderdg import Solver
    sc = inputs.SCENARIOS["adjoint_acoustic3d_n5_64"]
    ex = sc.extra
    steps = steps or sc.steps
    checkpoint = checkpoint or ex["checkpoint"]
    g = Solver.from_scenario(sc)
    c = torch.from_numpy(inputs.lognormal_speed(g.ncell, ex["c_mean"], ex["c_sigma"], ex["seed_c"])).cuda()
    g.set_material(c)
    dt = g.max_dt(sc.cfl)
    xs = inputs.source_point(sc, g.h)
    g.set_source(xs, ex["f0"], ex["t0"], ex["amp"])
    g.set_receivers(inputs.receivers_near(xs, g.h, ex["nrec"], 2.5, ex["seed_rec"]))
    Q0 = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    data = adj.record(g, torch.full_like(c, ex["c_mean"]), Q0, dt, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    adj.record(g, c, Q0, dt, steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0

    def gradient():
        cg = c.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = adj.misfit(cg, g, Q0, dt, steps, data, checkpoint)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        t0 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        return float(J.detach()), cg.grad, t_fwd, time.perf_counter() - t0

    J, grad, t_fwd, t_bwd = gradient()
    out = {"workload": "adjoint_acoustic3d_n5_64: 3-D acoustics N=5, 64^3 cells, %d steps, checkpoint %d, "
                       "64 receivers, Ricker f0=5, dt=%.6e" % (steps, checkpoint, dt),
           "forward_ms": 1e3 * t_fwd, "forward_plain_ms": 1e3 * t_plain, "backward_ms": 1e3 * t_bwd,
           "adjoint_over_forward": t_bwd / t_fwd, "misfit": J, "grad_norm": float(grad.norm())}
    if fd:
        rng = np.random.default_rng(7)
        dc = torch.from_numpy(rng.standard_normal(g.ncell)).cuda()
        eps = 1e-6 * float(c.norm()) / float(dc.norm())
        with torch.no_grad():
            jp = float(adj.misfit(c + eps * dc, g, Q0, dt, steps, data, checkpoint))
            jm = float(adj.misfit(c - eps * dc, g, Q0, dt, steps, data, checkpoint))
        fdv = (jp - jm) / (2 * eps)
        ad = float(grad @ dc)
        out.update({"fd_directional": fdv, "adjoint_directional": ad, "fd_rel_err": abs(fdv - ad) / abs(fdv),
                    "fd_tolerance": 1e-6})
    runs = []
    for p in mixed:
        g.set_precisions(p, p, "fp64")
        Jp, gp, tf, tb = gradient()
        runs.append({"predictor_volume": p, "forward_ms": 1e3 * tf, "backward_ms": 1e3 * tb,
                     "adjoint_over_forward": tb / tf, "backward_speedup_vs_fp64": t_bwd / tb,
                     "misfit_rel_err": abs(Jp - J) / abs(J),
                     "grad_rel_err": float((gp - grad).norm() / grad.norm())})
        print("adjoint %s: %.1f ms forward, %.1f ms backward, gradient rel err %.2e vs FP64" % (
            p, runs[-1]["forward_ms"], runs[-1]["backward_ms"], runs[-1]["grad_rel_err"]),
            file=sys.stderr, flush=True)
    g.set_precisions("fp64", "fp64", "fp64")
    if runs:
        out["mixed"] = runs
    g.close()
    return out


def sweep_runs(pde):
    """Precision settings (predictor, volume, flux) of the sweep: the 3-D Euler workload
    varies one kernel at a time and all three together; shallow water runs FP32 and BF16
    in the cell contractions (predictor and volume) and in every kernel."""
    if pde == "swe":
        return [("fp64", ("fp64",) * 3), ("predictor+volume=fp32", ("fp32", "fp32", "fp64")),
                ("all=fp32", ("fp32",) * 3), ("predictor+volume=bf16", ("bf16", "bf16", "fp64")),
                ("all=bf16", ("bf16",) * 3)]
    runs = [("fp64", ("fp64",) * 3)]
    for k, knob in enumerate(("predictor", "volume", "flux")):
        for p in ("fp32", "bf16", "fp16"):
            prec = ["fp64"] * 3
            prec[k] = p
            runs.append(("%s=%s" % (knob, p), tuple(prec)))
    runs += [("all=%s" % p, (p,) * 3) for p in ("fp32", "bf16", "fp16")]
    return runs


def sweep():
    """Per-kernel precision sweep on the 3-D Euler density wave (N=4, 48^3 cells, 200
    steps) and the 2-D shallow-water bump (N=6, 512^2 cells, 500 steps): for every
    setting the whole run's cell-DOF updates/s and the relative L2 error (eq. L2gauss)
    of the final state against the FP64 GPU run (parity-checked against the oracle) and,
    for Euler, against the exact solution."""
    import torch
    from paper_2504_06889_amd import inputs
    from paper_2504_06889_amd.aderdg import NonFiniteError, Solver
    out = {}
    for name in ("euler3d_n4_48", "swe2d_n6_512"):
        sc = inputs.SCENARIOS[name]
        g = Solver.from_scenario(sc)
        Q0 = torch.from_numpy(sc.initial_state(g.node_coords())).cuda()
        g.set_state(Q0)
        dt = g.max_dt(sc.cfl)
        W = torch.from_numpy(g.weights()).cuda()
        exact = None
        if sc.ic == "euler_density_wave":
            exact = torch.from_numpy(sc.initial_state(g.node_coords(), sc.steps * dt)).cuda()
        dof = g.ncell * g.S * g.V
        ref, runs = None, {}
        for label, prec in sweep_runs(sc.pde):
            g.set_precisions(*prec)
            g.set_state(Q0)
            g.time = 0.0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = {"precisions": dict(zip(("predictor", "volume", "flux"), prec))}
            try:
                g.step(dt, sc.steps)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                st = g.get_state(out=torch.empty(g.shape, dtype=torch.float64, device="cuda"))
            except NonFiniteError as e:
                r["error"] = "non-finite state: %s" % e
                runs[label] = r
                continue
            if ref is None:
                ref = st
            nref = l2(W, g.h, g.d, ref)
            r.update({"ms_per_step": 1e3 * el / sc.steps, "dof_per_s": dof * sc.steps / el,
                      "l2_rel_vs_fp64_gpu": l2(W, g.h, g.d, st, ref) / nref})
            if exact is not None:
                r["l2_rel_vs_exact"] = l2(W, g.h, g.d, st, exact) / l2(W, g.h, g.d, exact)
            runs[label] = r
            print("%s %s: %s" % (name, label, ", ".join("%s %.4g" % (k, v) for k, v in r.items()
                                                       if isinstance(v, float))), file=sys.stderr, flush=True)
        out[name] = {"steps": sc.steps, "dt": dt, "cells": g.ncell, "order": sc.order, "runs": runs}
        g.close()
        del ref, Q0, exact
        torch.cuda.empty_cache()
    return out


PAPER_RUNS = [("fp64", ("fp64",) * 3), ("predictor+volume=fp32", ("fp32", "fp32", "fp64")),
              ("flux=fp32", ("fp64", "fp64", "fp32")), ("predictor+volume=bf16", ("bf16", "bf16", "fp64")),
              ("predictor+volume=fp16", ("fp16", "fp16", "fp64")), ("all=fp32", ("fp32",) * 3),
              ("all=bf16", ("bf16",) * 3), ("all=fp16", ("fp16",) * 3),
              # every kernel and the stored state in the format (the paper's "all" columns)
              ("all+storage=fp32", ("fp32",) * 4), ("all+storage=bf16", ("bf16",) * 4),
              ("all+storage=fp16", ("fp16",) * 4)]


def paper_suite():
    """The paper's 2-D scenarios of its mixed-precision study (27^2 cells, order 5, run to
    t_end) with the state in FP64 and the predictor and volume contractions, the face
    kernels, or all of them in a lower format (the paper's one-kernel-at-a-time design),
    and with every kernel and the stored state in the format:
    the L2 error of eq. L2gauss against the interpolant of the exact solution at t_end,
    absolute (as the paper reports it) and relative, the relative L2 difference to the
    FP64 GPU run and, for the lake at rest, the largest spurious momentum."""
    import torch
    from paper_2504_06889_amd import inputs
    from paper_2504_06889_amd.aderdg import NonFiniteError, Solver
    out = {}
    for name, sc in inputs.PAPER_SUITE.items():
        g = Solver.from_scenario(sc)
        X = g.node_coords()
        Q0 = torch.from_numpy(sc.initial_state(X)).cuda()
        g.set_state(Q0)
        t_end = sc.extra["t_end"]
        nsteps = int(math.ceil(t_end / g.max_dt(sc.cfl)))
        dt = t_end / nsteps
        W = torch.from_numpy(g.weights()).cuda()
        exact = torch.from_numpy(sc.initial_state(X, t_end)).cuda()
        nex = l2(W, g.h, g.d, exact)
        ref, runs = None, {}
        for label, prec in PAPER_RUNS:
            g.set_precision("storage", prec[3] if len(prec) > 3 else "fp64")
            g.set_precisions(*prec[:3])
            g.set_state(Q0)
            g.time = 0.0
            r = {"precisions": dict(zip(("predictor", "volume", "flux", "storage"), tuple(prec) + ("fp64",) * (4 - len(prec))))}
            try:
                g.step(dt, nsteps)
                st = g.get_state(out=torch.empty(g.shape, dtype=torch.float64, device="cuda"))
            except NonFiniteError as e:
                r["error"] = "non-finite state: %s" % e
                runs[label] = r
                print("%s %s: non-finite" % (name, label), file=sys.stderr, flush=True)
                continue
            if ref is None:
                ref = st
            r["l2_vs_exact"] = l2(W, g.h, g.d, st, exact)
            r["l2_rel_vs_exact"] = r["l2_vs_exact"] / nex
            r["l2_rel_vs_fp64_gpu"] = l2(W, g.h, g.d, st, ref) / l2(W, g.h, g.d, ref)
            if sc.pde == "swe":
                r["max_abs_momentum"] = float(st[:, 1:3].abs().max())
            runs[label] = r
            print("%s %s: %s" % (name, label, ", ".join("%s %.3g" % (k, v) for k, v in r.items()
                                                       if isinstance(v, float))), file=sys.stderr, flush=True)
        out[name] = {"cells": list(sc.cells), "order": sc.order, "t_end": t_end, "steps": nsteps, "dt": dt,
                     "runs": runs}
        g.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="elastic3d_n5_64")
    ap.add_argument("--variants", default="fp64,fp32,bf16,fp16")
    ap.add_argument("--ck-variants", default="fp64,fp16",
                    help="precisions run with the Cauchy-Kowalevskaya predictor (linear PDEs), reported beside")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--sweep", action="store_true",
                    help="only run the per-kernel precision sweep on the Euler and shallow-water workloads")
    ap.add_argument("--paper-suite", action="store_true",
                    help="only run the paper's 2-D scenarios (27^2 cells, order 5) with lower-format kernels")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only run the adjoint configuration (forward and adjoint sweeps, FP64 and lower formats)")
    ap.add_argument("--adjoint-steps", type=int, default=0,
                    help="steps of the adjoint configuration (0: its own 200); with --adjoint-only")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (3 times), to scale HBM counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the step is not sharded across GPUs "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_06889_amd import inputs
    from paper_2504_06889_amd.aderdg import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        a_ = torch.ones(n, dtype=torch.float64, device="cuda")
        b_ = torch.empty_like(a_)
        for _ in range(3):
            b_.copy_(a_)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))
        return
    torch.cuda.set_device(0)
    if args.adjoint_only:
        steps = args.adjoint_steps or None
        txt = json.dumps({"adjoint": adjoint_bench(steps=steps, checkpoint=min(steps, 20) if steps else None,
                                                   fd=steps is None)})
        print(txt, flush=True)
        if args.out:
            with open(args.out, "w") as f:
                f.write(txt + "\n")
        return
    if args.sweep or args.paper_suite:
        txt = json.dumps({"sweep": sweep()} if args.sweep else {"paper_suite": paper_suite()})
        print(txt, flush=True)
        if args.out:
            with open(args.out, "w") as f:
                f.write(txt + "\n")
        return
    sc = inputs.SCENARIOS[args.workload]
    g = Solver.from_scenario(sc)
    print("workload %s: %d cells, N=%d, V=%d, S=%d" % (sc.name, g.ncell, sc.order, g.V, g.S), file=sys.stderr,
          flush=True)
    Q0h = sc.initial_state(g.node_coords())
    Q0 = torch.from_numpy(Q0h).cuda()
    del Q0h
    g.set_state(Q0)
    dt = g.max_dt(sc.cfl)
    W = torch.from_numpy(g.weights()).cuda()
    dof = g.ncell * g.S * g.V
    total_steps = args.warmup + args.steps
    T = total_steps * dt
    exact = torch.from_numpy(sc.initial_state(g.node_coords(), T)).cuda()
    nexact = l2(W, g.h, g.d, exact)

    runs = {}
    states = {}
    labels = [(p, "picard", p) for p in args.variants.split(",") if p]
    if sc.pde in ("acoustic", "elastic"):
        labels += [("ck_" + p, "ck", p) for p in args.ck_variants.split(",") if p]
    for label, kind, p in labels:
        prec = ("fp64", "fp64", "fp64") if p == "fp64" else (p, p, "fp64")
        g.set_predictor(kind)
        g.set_precisions(*prec)
        g.set_state(Q0)
        g.time = 0.0
        g.step(dt, args.warmup)
        torch.cuda.synchronize()
        g.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(dt, args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        tm = g.get_timing()
        g.set_timing(False)
        out = torch.empty(g.shape, dtype=torch.float64, device="cuda")
        g.get_state(out)
        p = label
        states[p] = out
        runs[p] = {"predictor": kind, "precisions": {"predictor": prec[0], "volume": prec[1], "flux": prec[2]},
                   "ms_per_step": 1e3 * el / args.steps, "dof_per_s": dof * args.steps / el,
                   "kernel_ms_per_step": (tm["predictor_ms"] + tm["corrector_ms"] + tm["fused_ms"]) / max(tm["steps"], 1),
                   "fused_kernel_ms": tm["fused_ms"] / max(tm["fused_launches"], 1),
                   "l2_rel_vs_exact": l2(W, g.h, g.d, out, exact) / nexact}
        print("%s: %.3f ms/step (kernels %.3f ms/step, fused corrector+predictor kernel %.3f ms)" % (
            p, runs[p]["ms_per_step"], runs[p]["kernel_ms_per_step"], runs[p]["fused_kernel_ms"]), file=sys.stderr,
            flush=True)
    # each predictor's lower-format runs against its own FP64 run; speed-ups against
    # the FP64 Picard path
    for kind, ref in (("picard", "fp64"), ("ck", "ck_fp64")):
        if ref not in states:
            continue
        nref = l2(W, g.h, g.d, states[ref])
        for p in runs:
            if runs[p]["predictor"] != kind:
                continue
            fmt = runs[p]["precisions"]["predictor"]
            runs[p]["l2_rel_vs_fp64_gpu"] = l2(W, g.h, g.d, states[p], states[ref]) / nref
            runs[p]["tolerance"] = TOL[fmt]
            runs[p]["within_tolerance"] = bool(runs[p]["l2_rel_vs_fp64_gpu"] <= TOL[fmt])
            if "fp64" in runs:
                runs[p]["speedup_vs_fp64"] = runs["fp64"]["ms_per_step"] / runs[p]["ms_per_step"]

    # roofline of the dominant kernel (the fused corrector + predictor) for each variant
    traffic = measured_traffic() if args.workload == "elastic3d_n5_64" else {}
    I = g.iters
    mf, v64, fl = predictor_flops(sc.pde, sc.dim, sc.order, g.V, I)
    v64 += corrector_flops(sc.dim, sc.order, g.V)
    for p in runs:
        if runs[p]["predictor"] != "picard":
            continue  # the roofline counts are the Picard predictor's
        t = runs[p]["fused_kernel_ms"] * 1e-3
        total = (mf + v64 + fl) * g.ncell
        if p == "fp64":
            ideal = total / PEAK["fp64"]
            bound = "alu"
        else:
            t_m = mf * g.ncell / PEAK["mfma_" + p]
            t_v = v64 * g.ncell / PEAK["fp64"] + fl * g.ncell / PEAK["fp32_valu"]
            ideal = t_m + t_v
            bound = "mfma" if t_m > t_v else "alu"
        hbm = fused_bytes(sc.dim, sc.order, g.V, 8, sc.pde in ("acoustic", "elastic")) * g.ncell
        runs[p]["roofline"] = {
            "bound": bound, "achieved": total / t / 1e12, "peak": total / ideal / 1e12, "unit": "TFLOP/s",
            "frac": ideal / t, "traffic": traffic.get(p),
            "flops_per_launch": total, "mfma_flops_per_launch": (mf * g.ncell if p != "fp64" else 0),
            "hbm_bytes_per_launch": hbm, "hbm_GBps": hbm / t / 1e9}

    g.close()
    del states, Q0, exact
    torch.cuda.empty_cache()
    head = HEADLINE if HEADLINE in runs else [p for p in runs if runs[p]["predictor"] == "picard"][-1]
    r = runs[head]
    line = {
        "metric": "cell-DOF updates/s, mixed vs FP64 GPU at stated L2 error; adjoint/forward time",
        "value": r["dof_per_s"], "unit": "cell-DOF updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "%s-mfma+f64" % head if head != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: 3-D elastic waves, N=5, 64^3 periodic cells, planar P+S wave, %s, "
                               "Picard time operator, averages, flux/corrector and state FP64, "
                               "C_CFL=%.2f, dt=%.6e" % (
                                   sc.name, "all contractions FP64 on the vector ALU" if head == "fp64" else
                                   "predictor+volume contractions in %s on matrix cores (FP32 accumulate)" % head,
                                   sc.cfl, dt),
                   "cells": g.ncell, "order": sc.order, "dof_per_step": dof, "picard_iters": I},
        "roofline": r["roofline"],
        "speedup_vs_fp64": r.get("speedup_vs_fp64"),
        "l2_rel_vs_fp64_gpu": r.get("l2_rel_vs_fp64_gpu"), "tolerance": TOL.get(head),
        "runs": runs,
    }
    if not args.no_adjoint:
        line["adjoint"] = adjoint_bench()
        print("adjoint: %.1f ms forward, %.1f ms backward, ratio %.2f, fd rel err %.2e" % (
            line["adjoint"]["forward_ms"], line["adjoint"]["backward_ms"], line["adjoint"]["adjoint_over_forward"],
            line["adjoint"].get("fd_rel_err", float("nan"))), file=sys.stderr, flush=True)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(sc, args.cpu_seconds)
    txt = json.dumps(line)
    print(txt, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(txt + "\n")


if __name__ == "__main__":
    main()
