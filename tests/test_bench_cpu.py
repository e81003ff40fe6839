"""Host-side checks of bench.py: the one-GPU contract, the precision sweep's
settings and the rule that measured traffic is only reported for the profiled
kernel sources."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_sweep_settings():
    eu = bench.sweep_runs("euler")
    assert len(eu) == 13 and eu[0] == ("fp64", ("fp64",) * 3)
    labels = [k for k, _ in eu]
    assert len(set(labels)) == 13
    for k, prec in eu[1:]:
        knob, p = k.split("=")
        if knob == "all":
            assert prec == (p, p, p)
        else:
            i = ("predictor", "volume", "flux").index(knob)
            assert prec[i] == p and all(prec[m] == "fp64" for m in range(3) if m != i)
    swe = dict(bench.sweep_runs("swe"))
    assert swe["predictor+volume=bf16"] == ("bf16", "bf16", "fp64") and swe["all=fp32"] == ("fp32",) * 3


def test_profile_values_only_for_profiled_sources(tmp_path):
    src = os.path.join(ROOT, "profiles", "k_predictor_elastic3d_n5_64_hbm_traffic.md")
    if not os.path.exists(src):
        pytest.skip("no traffic summary committed")
    text = open(src).read()
    fake = tmp_path / "traffic.md"
    fake.write_text(text.replace("kernel-source-sha256: ", "kernel-source-sha256: 0"))
    assert bench.profile_values(str(fake), "traffic-bytes-per-launch") == {}
    fake.write_text("\n".join(l if not l.strip().startswith("kernel-source-sha256:")
                              else "    kernel-source-sha256: " + bench.kernel_source_hash()
                              for l in text.split("\n")))
    t = bench.profile_values(str(fake), "traffic-bytes-per-launch")
    assert {"fp64", "fp32", "bf16", "fp16"} <= set(t) and all(v > 0 for v in t.values())
    # the other entries are runs with the state stored in a narrower format
    for k in set(t) - {"fp64", "fp32", "bf16", "fp16"}:
        p, st = k.split("+storage_")
        assert p in ("fp64", "fp32", "bf16", "fp16") and st in ("fp32", "bf16", "fp16")
        assert t[k] < t[p]


def test_roofline_fractions_of_published_peaks():
    """The binding fraction is the largest of HBM bytes / 8 TB/s, matrix-core flops /
    the format's dense peak and FP64 vector flops / 78.6 TFLOP/s; each is recomputable
    from the counts and the launch time."""
    d, N, V, I, ncell, t = 3, 5, 9, 6, 64 ** 3, 16.7e-3
    mf, v64, fl = bench.predictor_flops("elastic", d, N, V, I)
    v64 += bench.corrector_flops(d, N, V)
    r = bench.roofline("elastic", d, N, V, I, ncell, t, "fp16", True, traffic=2e10, mfma_busy=3.6e9)
    hbm = bench.fused_bytes(d, N, V, 8, True) * ncell
    assert abs(r["fractions"]["hbm"] - hbm / t / 8e12) < 1e-12
    assert abs(r["fractions"]["mfma_fp16"] - mf * ncell / t / 2.5e15) < 1e-12
    assert abs(r["fractions"]["fp64_valu"] - v64 * ncell / t / 78.6e12) < 1e-12
    key = max(r["fractions"], key=r["fractions"].get)
    assert abs(r["frac"] - r["fractions"][key]) < 1e-12
    assert abs(r["achieved"] / r["peak"] - r["frac"]) < 1e-12
    assert abs(r["mfma_util"] - 3.6e9 / (t * 2.4e9 * 1024)) < 1e-12
    r64 = bench.roofline("elastic", d, N, V, I, ncell, 33.6e-3, "fp64", True)
    assert r64["bound"] == "alu" and r64["unit"] == "TFLOP/s"
    assert abs(r64["achieved"] * 1e12 - (mf + v64 + fl) * ncell / 33.6e-3) < 1e-3 * r64["achieved"] * 1e12
