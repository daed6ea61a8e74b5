"""The committed bench line (profiles/bench_sphere1m_p6.json) against the
output contract of bench.py, and the one-GPU refusal (no GPU needed).

The line's roofline must follow from its own figures: achieved = algorithmic
flops per M2L launch / the launch's average time, frac = achieved / peak, with
the FP32 MFMA peak of the MI355X (157.3 TFLOP/s); the same for every stage in
stage_roofline, against the peak its bound names; the value is the mean of the
timed steps; and the CPU baseline is the oracle's.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..")
LINE = os.path.join(ROOT, "profiles", "bench_sphere1m_p6.json")
PEAKS = {("mfma", "TFLOP/s"): 157.3, ("alu", "TFLOP/s"): 157.3, ("hbm", "GB/s"): 8000.0}


@pytest.fixture(scope="module")
def line():
    with open(LINE) as f:
        return json.load(f)


def test_required_fields(line):
    for key, typ in (("metric", str), ("value", float), ("unit", str), ("n_gpus", int), ("steps", int),
                     ("warmup", int), ("ms_per_step", float), ("higher_is_better", bool), ("scaling", str),
                     ("dtype", str), ("data", str), ("config", dict), ("roofline", dict),
                     ("cpu_baseline", dict)):
        assert isinstance(line[key], typ), key
    assert line["n_gpus"] == 1 and line["unit"] == "ms" and line["higher_is_better"] is False
    assert line["value"] == line["ms_per_step"] == line["timing_ms"]["mean"]
    assert line["timing_ms"]["min"] <= line["timing_ms"]["median"] <= line["timing_ms"]["max"]
    assert line["vs_baseline"] is None
    assert "workload" in line["config"] and "model" not in line["config"]
    assert line["config"]["n"] == 1 << 20 and line["config"]["p"] == 6 and line["config"]["leaf_size"] == 64


def test_roofline_follows_from_its_figures(line):
    r = line["roofline"]
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == PEAKS[("mfma", "TFLOP/s")]
    # 2 k^2 flop per V-list pair: k = 119, 4,216,540 pairs
    assert r["flops_per_launch"] == 2 * line["config"]["k"] ** 2 * line["config"]["v_pairs"]
    assert r["achieved"] == pytest.approx(r["flops_per_launch"] / (r["avg_launch_ms"] * 1e-3) / 1e12, rel=2e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-3)
    assert r["avg_launch_ms"] == pytest.approx(line["stage_ms"]["m2l"], abs=1e-3)
    # the committed kernel trace agrees with the events to a few per cent
    assert r["trace"]["avg_launch_ms"] == pytest.approx(r["avg_launch_ms"], rel=0.05)
    # calibrated HBM traffic per launch, at least the algorithmic bytes
    assert r["traffic"] is None or r["traffic"] > 1e8


def test_stage_rooflines_follow_from_their_figures(line):
    for name, s in line["stage_roofline"].items():
        assert s["peak"] == PEAKS[(s["bound"], s["unit"])], name
        scale = 1e12 if s["unit"] == "TFLOP/s" else 1e9
        assert s["achieved"] == pytest.approx(s["work_per_apply"] / (s["ms"] * 1e-3) / scale, rel=5e-3), name
        assert s["frac"] == pytest.approx(s["achieved"] / s["peak"], abs=1e-3), name


def test_cpu_baseline_is_the_oracle(line):
    c = line["cpu_baseline"]
    assert c["kind"] == "oracle" and c["unit"] == line["unit"] and c["cores"] >= 1 and c["value"] > 0
    assert c["sample"]


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0 and "one GPU" in r.stdout + r.stderr
