"""Throughput of the ADER-DG time step on one MI355X.

Workload: 3-D linear elastic waves (9 variables), order N = 5 (6 Gauss-Legendre
nodes per dimension), 64^3 periodic cells on the unit cube, rho = 2.7,
cp = 6.0, cs = 3.464, planar P + S wave; C_CFL = 0.5 in
dt = C h / (d (2N+1) lambda_max).  One step = predictor (Picard iteration),
face projection, volume integral, Rusanov flux and corrector over all cells.

The same K steps are timed for the all-FP64 path and for the predictor and
volume contractions in FP32 (vector ALU), BF16 and FP16 (matrix cores), with
FP32 accumulation; Picard time operator, time averages, flux/corrector and
state in FP64.  `value` is the FP16 variant's cell-DOF updates/s (DOF = cells * n^3 * 9
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

# MI355X published peaks: FP64 vector (= FP64 matrix) 78.6 TFLOP/s, FP32 157.3
# TFLOP/s (vector, packed; dense matrix), dense BF16/FP16 matrix 2.5 PFLOP/s,
# HBM3E 8 TB/s; 1024 SIMDs (256 CUs) at 2.4 GHz.
PEAK = {"fp64": 78.6e12, "fp32_valu": 157.3e12, "mfma_bf16": 2.5e15, "mfma_fp16": 2.5e15, "hbm": 8.0e12}
CLOCK_HZ = 2.4e9
SIMDS = 1024
TOL = {"fp64": 1e-10, "fp32": 1e-6, "fp16": 1e-3, "bf16": 1e-2}
HEADLINE = "fp16"


def flux_flops(pde, d):
    """Flops of one pointwise flux F_j (one direction, one node)."""
    return {"acoustic": 2, "elastic": 8 if d == 3 else 5, "euler": 3 * d + 7, "swe": 3}[pde]


def predictor_flops(pde, d, N, V, I):
    """Algorithmic flops per cell of one predictor launch (sum-factorised, no
    padding): returns (contraction flops -- on the matrix cores in BF16/FP16, on
    the vector ALU in FP32 and FP64 --, FP64 vector flops, pointwise-flux flops)."""
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


def fused_bytes(d, N, V, face_bytes, q_only, state_bytes=8):
    """HBM bytes per cell of one fused launch (corrector of the previous step +
    predictor): Q* read and written (state_bytes per value: 8 for FP64 storage, 4 or 2
    for a narrower storage format), the previous face data of the cell and of its
    neighbours read, the new face data written.  For a linear PDE with FP64 faces only
    the projected q is stored."""
    n = N + 1
    S = n ** d
    F = S // n
    faces = 2 * d * V * F * face_bytes * (1 if q_only else 2)
    return 2 * S * V * state_bytes + 2 * faces + faces


# Sources that determine the machine code of k_predictor for this workload.
KERNEL_SOURCES = ("paper_2504_06889_amd/csrc/common.h", "paper_2504_06889_amd/csrc/kernels.h",
                  "paper_2504_06889_amd/csrc/registry.h", "paper_2504_06889_amd/csrc/inst_elastic3.hip",
                  "paper_2504_06889_amd/csrc/inst_euler.hip", "paper_2504_06889_amd/csrc/inst_swe.hip",
                  "paper_2504_06889_amd/build.py")


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


def profile_values(path, tag):
    """Values `tag <variant>: <number>` of a committed rocprofv3 summary under
    profiles/, or {} when the kernel sources have changed since it was taken (its
    kernel-source-sha256 line no longer matches)."""
    path = os.path.join(ROOT, path)
    if not os.path.exists(path):
        return {}
    out, ok = {}, False
    with open(path) as fh:
        for line in fh:
            t = line.strip()
            if t.startswith("kernel-source-sha256:"):
                ok = t.split(":", 1)[1].strip() == kernel_source_hash()
            elif t.startswith(tag + " "):
                key, val = t[len(tag):].split(":")
                out[key.strip()] = float(val)
    return out if ok else {}


def measured_traffic(workload="elastic3d_n5_64"):
    """Per-launch HBM bytes of the fused kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (scaled by a plain copy's counter readings)."""
    return profile_values("profiles/k_predictor_%s_hbm_traffic.md" % workload, "traffic-bytes-per-launch")


def measured_mfma_busy(workload="elastic3d_n5_64"):
    """SQ_VALU_MFMA_BUSY_CYCLES per launch of the fused kernel (summed over SIMDs)."""
    return profile_values("profiles/k_predictor_%s_sq_counters.md" % workload, "mfma-busy-cycles-per-launch")


def roofline(pde, d, N, V, I, ncell, t, prec, q_only, traffic=None, mfma_busy=None, state_bytes=8):
    """Roofline entry of one fused launch (corrector of the previous step + predictor)
    taking t seconds: the achieved fraction of each published peak the launch's
    algorithmic work touches -- HBM bytes / 8 TB/s, the contraction flops / the
    format's dense matrix peak (BF16, FP16) or the FP32 vector peak (FP32, whose
    contractions run on the vector ALU), the FP64 vector flops / 78.6 TFLOP/s (in
    FP64 every flop) -- and the binding one (largest fraction) as
    bound/achieved/peak/frac.  design_bound: the launch time if every unit ran at its
    peak at once (max over units) and, for comparison, the blended sum of the unit
    times.  traffic: HBM bytes per launch measured with rocprofv3 counters (or None);
    mfma_busy: SQ_VALU_MFMA_BUSY_CYCLES per launch summed over SIMDs (or None)."""
    mf, v64, fl = predictor_flops(pde, d, N, V, I)
    v64 += corrector_flops(d, N, V)
    hbm = fused_bytes(d, N, V, 8, q_only, state_bytes) * ncell
    total = (mf + v64 + fl) * ncell
    fr = {"hbm": hbm / t / PEAK["hbm"]}
    times = {"hbm": hbm / PEAK["hbm"]}
    if prec == "fp64":
        fr["fp64_valu"] = total / t / PEAK["fp64"]
        times["fp64_valu"] = total / PEAK["fp64"]
    else:
        ck = "fp32_valu" if prec == "fp32" else "mfma_" + prec
        fr[ck] = mf * ncell / t / PEAK[ck]
        fr["fp64_valu"] = v64 * ncell / t / PEAK["fp64"]
        times[ck] = mf * ncell / PEAK[ck]
        times["fp64_valu"] = v64 * ncell / PEAK["fp64"] + fl * ncell / PEAK["fp32_valu"]
    key = max(fr, key=fr.get)
    if key == "hbm":
        achieved, peak, unit = hbm / t / 1e9, PEAK["hbm"] / 1e9, "GB/s"
        bound = "hbm"
    elif key.startswith("mfma") or key == "fp32_valu":
        achieved, peak, unit = mf * ncell / t / 1e12, PEAK[key] / 1e12, "TFLOP/s"
        bound = "mfma" if key.startswith("mfma") else "alu"
    else:
        work = total if prec == "fp64" else v64 * ncell
        achieved, peak, unit = work / t / 1e12, PEAK["fp64"] / 1e12, "TFLOP/s"
        bound = "alu"
    out = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
           "traffic": traffic, "fractions": fr,
           "flops_per_launch": total, "mfma_flops_per_launch": (mf * ncell if prec in ("bf16", "fp16") else 0),
           "fp64_flops_per_launch": total if prec == "fp64" else v64 * ncell,
           "hbm_bytes_per_launch": hbm, "launch_ms": 1e3 * t,
           "design_bound": {"max_unit_ms": 1e3 * max(times.values()), "blended_ms": 1e3 * sum(times.values()),
                            "frac_of_max_unit": max(times.values()) / t}}
    if traffic:
        out["traffic_GBps"] = traffic / t / 1e9
    if mfma_busy is not None:
        out["mfma_util"] = mfma_busy / (t * CLOCK_HZ * SIMDS)
    return out


def l2(W, h, d, A, B=None):
    import torch
    diff = A if B is None else A - B
    return float(torch.sqrt((diff * diff * W[None, None, :]).sum() * h ** d))


def cpu_model():
    """Host CPU model name (from /proc/cpuinfo) and the number of logical CPUs."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def _time_oracle(o, dt, seconds):
    o.step(0.0, dt)  # warm-up
    steps, t0 = 0, time.perf_counter()
    while True:
        o.step(steps * dt, dt)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 2000:
            return steps, el


def cpu_baseline(sc, seconds=12.0, cells=8):
    """The FP64 oracle on a periodic cells^3 sub-grid of the same problem (same
    order, cell size and per-cell work), timed on the host cores: all threads
    (value, cores), then one thread for half the time."""
    import oracle
    h = (sc.hi[0] - sc.lo[0]) / sc.cells[0]
    o = oracle.Oracle(sc.dim, sc.order, (cells,) * sc.dim, sc.lo, tuple(sc.lo[j] + cells * h for j in range(sc.dim)),
                      sc.pde, sc.params)
    o.set_state(sc.initial_state(o.node_coords()))
    dt = o.max_dt(sc.cfl)
    dof = o.ncell * o.S * o.V
    cores = oracle.num_threads()
    steps, el = _time_oracle(o, dt, seconds)
    oracle.set_num_threads(1)
    steps1, el1 = _time_oracle(o, dt, 0.5 * seconds)
    oracle.set_num_threads(cores)
    model, ncpu = cpu_model()
    return {"value": dof * steps / el, "unit": "cell-DOF updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d FP64 oracle steps of the same problem on a periodic %d^3-cell sub-grid "
                      "(%d cells, same order and cell size), %.1f s on %d threads; one thread: %d steps, %.1f s" % (
                          steps, cells, o.ncell, el, cores, steps1, el1),
            "one_thread": {"value": dof * steps1 / el1, "cores": 1},
            "cpu_model": model, "logical_cpus": ncpu}


def golden(name):
    """The full-length FP64 oracle reference of a workload (tests/golden, written by
    tests/golden/make_fullsize.py with the oracle only), or None."""
    path = os.path.join(ROOT, "tests", "golden", "fullsize_%s.npz" % name)
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def vs_oracle(ref, B, W):
    """Sampled-cell comparison with the oracle reference: relative L2 (eq. L2gauss
    weights) over the sampled cells, and the largest |B - A| over each variable's
    largest |A| (both over the sampled cells)."""
    A = ref["Q"]
    w = W[None, None, :]
    rel = float(np.sqrt(((B - A) ** 2 * w).sum() / (A ** 2 * w).sum()))
    scale = np.abs(A).max(axis=(0, 2))
    elem = float((np.abs(B - A).max(axis=(0, 2)) / np.where(scale > 0, scale, 1.0)).max())
    return {"l2_rel_vs_fp64_oracle": rel, "max_rel_vs_fp64_oracle": elem, "cells_sampled": int(A.shape[0]),
            "steps": int(ref["nsteps"])}


def accuracy_run(g, sc, Q0, ref):
    """The workload's own number of steps from the initial state at the oracle
    reference's dt, compared with the reference at its sampled cells."""
    import torch
    g.set_state(Q0)
    g.time = 0.0
    g.step(float(ref["dt"]), int(ref["nsteps"]))
    ids = torch.from_numpy(ref["ids"]).cuda()
    st = g.get_state(out=torch.empty(g.shape, dtype=torch.float64, device="cuda"))
    B = st.index_select(0, ids).cpu().numpy()
    del st
    return vs_oracle(ref, B, g.weights())


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


def workload_runs(name):
    """One workload's precision settings (sweep_runs), each run for the workload's
    own number of steps from the initial state and timed whole: ms/step, cell-DOF
    updates/s, the fused kernel's time per launch (HIP events) and its roofline, the
    relative L2 error (eq. L2gauss) of the final state against the FP64 GPU run, the
    exact solution (density wave) and, at the sampled cells of the full-length FP64
    oracle reference (when present), against the oracle."""
    import torch
    from paper_2504_06889_amd import inputs
    from paper_2504_06889_amd.aderdg import NonFiniteError, Solver
    sc = inputs.SCENARIOS[name]
    g = Solver.from_scenario(sc)
    Q0 = torch.from_numpy(sc.initial_state(g.node_coords())).cuda()
    g.set_state(Q0)
    dt = g.max_dt(sc.cfl)
    ref_o = golden(name)
    if ref_o is not None and abs(float(ref_o["dt"]) - dt) <= 1e-14 * dt:
        dt = float(ref_o["dt"])  # the reference's dt (equal up to rounding)
    else:
        ref_o = None
    W = torch.from_numpy(g.weights()).cuda()
    Wn = g.weights()
    exact = None
    if sc.ic == "euler_density_wave":
        exact = torch.from_numpy(sc.initial_state(g.node_coords(), sc.steps * dt)).cuda()
    dof = g.ncell * g.S * g.V
    traffic, busy = measured_traffic(name), measured_mfma_busy(name)
    ref, runs = None, {}
    for label, prec in sweep_runs(sc.pde):
        g.set_precisions(*prec)
        g.set_state(Q0)
        g.time = 0.0
        r = {"precisions": dict(zip(("predictor", "volume", "flux"), prec))}
        torch.cuda.synchronize()
        g.set_timing(True)
        t0 = time.perf_counter()
        try:
            g.step(dt, sc.steps)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            tm = g.get_timing()
            st = g.get_state(out=torch.empty(g.shape, dtype=torch.float64, device="cuda"))
        except NonFiniteError as e:
            g.set_timing(False)
            r["error"] = "non-finite state: %s" % e
            runs[label] = r
            print("%s %s: non-finite" % (name, label), file=sys.stderr, flush=True)
            continue
        g.set_timing(False)
        if ref is None:
            ref = st
        nref = l2(W, g.h, g.d, ref)
        fused = tm["fused_ms"] / max(tm["fused_launches"], 1)
        r.update({"ms_per_step": 1e3 * el / sc.steps, "dof_per_s": dof * sc.steps / el, "fused_kernel_ms": fused,
                  "l2_rel_vs_fp64_gpu": l2(W, g.h, g.d, st, ref) / nref})
        if exact is not None:
            r["l2_rel_vs_exact"] = l2(W, g.h, g.d, st, exact) / l2(W, g.h, g.d, exact)
        if ref_o is not None:
            ids = torch.from_numpy(ref_o["ids"]).cuda()
            r.update(vs_oracle(ref_o, st.index_select(0, ids).cpu().numpy(), Wn))
        # roofline of the fused kernel, its contraction flops counted in the
        # predictor's format (the volume contraction is a few per cent of them)
        key = "fp64" if prec == ("fp64",) * 3 else label
        r["roofline"] = roofline(sc.pde, sc.dim, sc.order, g.V, g.iters, g.ncell, fused * 1e-3, prec[0],
                                 sc.pde in ("acoustic", "elastic") and prec[2] == "fp64", traffic.get(key),
                                 busy.get(key))
        runs[label] = r
        print("%s %s: %s" % (name, label, ", ".join("%s %.4g" % (k, v) for k, v in r.items()
                                                   if isinstance(v, float))), file=sys.stderr, flush=True)
    out = {"workload": "%s: %s, N=%d, %s cells, %d steps, C_CFL=%.2f, dt=%.6e" % (
               name, sc.pde, sc.order, "x".join(map(str, sc.cells)), sc.steps, sc.cfl, dt),
           "steps": sc.steps, "dt": dt, "cells": g.ncell, "order": sc.order, "dof_per_step": dof,
           "oracle_reference": ref_o is not None, "runs": runs}
    g.close()
    del ref, Q0, exact
    torch.cuda.empty_cache()
    return out


def sweep():
    """Per-kernel precision sweep on the 3-D Euler density wave (N=4, 48^3 cells, 200
    steps) and the 2-D shallow-water bump (N=6, 512^2 cells, 500 steps)."""
    return {name: workload_runs(name) for name in ("euler3d_n4_48", "swe2d_n6_512")}


PAPER_RUNS = [("fp64", ("fp64",) * 3), ("predictor+volume=fp32", ("fp32", "fp32", "fp64")),
              ("flux=fp32", ("fp64", "fp64", "fp32")), ("predictor+volume=bf16", ("bf16", "bf16", "fp64")),
              ("predictor+volume=fp16", ("fp16", "fp16", "fp64")), ("all=fp32", ("fp32",) * 3),
              ("all=bf16", ("bf16",) * 3), ("all=fp16", ("fp16",) * 3),
              # every kernel and the stored state in the format (the paper's "all" columns)
              ("all+storage=fp32", ("fp32",) * 4), ("all+storage=bf16", ("bf16",) * 4),
              ("all+storage=fp16", ("fp16",) * 4)]


def paper_table_runs():
    """Settings (predictor, volume, flux, storage) of the paper's two tables of one
    kernel changed against a base (Sec. 7), mapped to this library's knobs: the
    paper's "Picard" kernel is PREDICTOR (the Picard contractions), its "predictor"
    kernel PREDICTOR + VOLUME (its fused predictor computes the volume integral), its
    "corrector" FLUX, "all" every kernel.
      fp32-storage table: state and every kernel FP32, one kernel (or all) in BF16
        or FP16;
      higher-fp64 table: state and every kernel in a base format (BF16, FP16,
        FP32), one kernel (or all kernels) in FP64."""
    def one(kernel, p, base):
        pr, vo, fl = base, base, base
        if kernel == "Picard":
            pr = p
        elif kernel == "predictor":
            pr = vo = p
        elif kernel == "corrector":
            fl = p
        elif kernel == "all":
            pr = vo = fl = p
        return (pr, vo, fl, base)
    runs = [("storage_fp32:reference", ("fp32",) * 4)]
    for p in ("bf16", "fp16"):
        for k in ("Picard", "predictor", "corrector", "all"):
            runs.append(("storage_fp32:%s=%s" % (k, p), one(k, p, "fp32")))
    for base in ("bf16", "fp16", "fp32"):
        runs.append(("base_%s:reference" % base, (base,) * 4))
        for k in ("Picard", "predictor", "corrector", "all"):
            runs.append(("base_%s:%s=fp64" % (base, k), one(k, "fp64", base)))
    return runs


def paper_suite_runs(sc, settings, label_prefix=""):
    """Run the settings (predictor, volume, flux[, storage]) of a 2-D scenario to t_end:
    the L2 error of eq. L2gauss against the interpolant of the exact solution at t_end,
    absolute (as the paper reports it) and relative, the relative L2 difference to the
    FP64 GPU run and, for the lake at rest, the largest spurious momentum."""
    import torch
    from paper_2504_06889_amd.aderdg import NonFiniteError, Solver
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
    for label, prec in [("fp64", ("fp64",) * 4)] + list(settings):
        prec = tuple(prec) + ("fp64",) * (4 - len(prec))
        g.set_precision("storage", prec[3])
        g.set_precisions(*prec[:3])
        g.set_state(Q0)
        g.time = 0.0
        r = {"precisions": dict(zip(("predictor", "volume", "flux", "storage"), prec))}
        try:
            g.step(dt, nsteps)
            st = g.get_state(out=torch.empty(g.shape, dtype=torch.float64, device="cuda"))
        except NonFiniteError as e:
            r["error"] = "non-finite state: %s" % e
            runs[label] = r
            print("%s %s: non-finite" % (sc.name, label), file=sys.stderr, flush=True)
            continue
        if ref is None:
            ref = st
        r["l2_vs_exact"] = l2(W, g.h, g.d, st, exact)
        r["l2_rel_vs_exact"] = r["l2_vs_exact"] / nex
        r["l2_rel_vs_fp64_gpu"] = l2(W, g.h, g.d, st, ref) / l2(W, g.h, g.d, ref)
        if sc.pde == "swe":
            r["max_abs_momentum"] = float(st[:, 1:3].abs().max())
        runs[label] = r
        print("%s %s: %s" % (sc.name, label, ", ".join("%s %.3g" % (k, v) for k, v in r.items()
                                                      if isinstance(v, float))), file=sys.stderr, flush=True)
    g.close()
    return {"cells": list(sc.cells), "order": sc.order, "t_end": t_end, "steps": nsteps, "dt": dt, "runs": runs}


def paper_suite():
    """The paper's 2-D scenarios of its mixed-precision study (27^2 cells, order 5, run to
    t_end): the state in FP64 with the predictor and volume contractions, the face
    kernels, or all of them in a lower format (the paper's one-kernel-at-a-time
    design) and every kernel and the stored state in the format; the settings of the
    paper's FP32-storage table and of its table of one kernel in FP64 on a lower base;
    and the two Euler scenarios on 81^2 cells with an FP32 base and one kernel in FP64
    (the paper's finer-grid table)."""
    from paper_2504_06889_amd import inputs
    out = {}
    table = paper_table_runs()
    for name, sc in inputs.PAPER_SUITE.items():
        out[name] = paper_suite_runs(sc, PAPER_RUNS[1:] + table)
    for name in ("euler2d_n5_27_bell", "euler2d_n5_27_vortex"):
        sc = inputs.PAPER_SUITE[name].with_cells((81, 81))
        fine = [(k, p) for k, p in table if k.startswith("base_fp32:")]
        out[name.replace("_27_", "_81_")] = paper_suite_runs(sc, fine)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="elastic3d_n5_64")
    ap.add_argument("--variants", default="fp64,fp32,bf16,fp16")
    ap.add_argument("--storage", default="fp64", choices=("fp64", "fp32", "bf16", "fp16"),
                    help="storage format of the state in the timed runs of the headline workload")
    ap.add_argument("--ck-variants", default="fp64,fp16",
                    help="precisions run with the Cauchy-Kowalevskaya predictor (linear PDEs), reported beside")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the 3-D Euler and 2-D shallow-water precision runs")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the full-length runs compared with the FP64 oracle reference")
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
        g.set_precision("storage", args.storage)
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
        runs[p] = {"predictor": kind, "precisions": {"predictor": prec[0], "volume": prec[1], "flux": prec[2],
                                                     "storage": args.storage},
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

    # roofline of the dominant kernel (the fused corrector + predictor) for each
    # Picard variant (the counts are the Picard predictor's)
    traffic, busy = measured_traffic(args.workload), measured_mfma_busy(args.workload)
    for p in runs:
        if runs[p]["predictor"] != "picard":
            continue
        st = args.storage
        runs[p]["roofline"] = roofline(sc.pde, sc.dim, sc.order, g.V, g.iters, g.ncell,
                                       runs[p]["fused_kernel_ms"] * 1e-3, p, sc.pde in ("acoustic", "elastic"),
                                       traffic.get(p if st == "fp64" else "%s+storage_%s" % (p, st)),
                                       busy.get(p) if st == "fp64" else None,
                                       {"fp64": 8, "fp32": 4}.get(st, 2))

    # the workload's own number of steps from the initial state, each variant
    # against the full-length FP64 oracle reference at its sampled cells
    ref_o = golden(args.workload)
    if ref_o is not None and not args.no_accuracy:
        for label, kind, p in labels:
            prec = ("fp64", "fp64", "fp64") if p == "fp64" else (p, p, "fp64")
            g.set_predictor(kind)
            g.set_precisions(*prec)
            acc = accuracy_run(g, sc, Q0, ref_o)
            acc["tolerance"] = TOL[p]
            acc["within_tolerance"] = bool(acc["l2_rel_vs_fp64_oracle"] <= TOL[p])
            runs[label]["vs_fp64_oracle"] = acc
            print("%s vs FP64 oracle after %d steps: rel L2 %.3e, max rel %.3e" % (
                label, acc["steps"], acc["l2_rel_vs_fp64_oracle"], acc["max_rel_vs_fp64_oracle"]),
                file=sys.stderr, flush=True)
        g.set_predictor("picard")

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
                   "cells": g.ncell, "order": sc.order, "dof_per_step": dof, "picard_iters": g.iters},
        "roofline": r["roofline"],
        "speedup_vs_fp64": r.get("speedup_vs_fp64"),
        "l2_rel_vs_fp64_gpu": r.get("l2_rel_vs_fp64_gpu"), "tolerance": TOL.get(head),
        "l2_rel_vs_fp64_oracle": r.get("vs_fp64_oracle", {}).get("l2_rel_vs_fp64_oracle"),
        "runs": runs,
    }
    if not args.no_workloads:
        line["workloads"] = {}
        for name in ("euler3d_n4_48", "swe2d_n6_512"):
            line["workloads"][name] = workload_runs(name)
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
