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


def test_traffic_only_for_profiled_sources(tmp_path, monkeypatch):
    src = os.path.join(ROOT, bench.TRAFFIC_FILE)
    if not os.path.exists(src):
        pytest.skip("no traffic summary committed")
    text = open(src).read()
    fake = tmp_path / "traffic.md"
    fake.write_text(text.replace("kernel-source-sha256: ", "kernel-source-sha256: 0"))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(fake))
    assert bench.measured_traffic() == {}
    fake.write_text("\n".join(l if not l.strip().startswith("kernel-source-sha256:")
                              else "    kernel-source-sha256: " + bench.kernel_source_hash()
                              for l in text.split("\n")))
    t = bench.measured_traffic()
    assert set(t) == {"fp64", "fp32", "bf16", "fp16"} and all(v > 0 for v in t.values())
