"""Host logic of the benchmark script (no GPU): the one-GPU guard, the
stale-counter check and the time-to-1% extrapolation."""

import json
import math
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
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_code_only_ignores_comments_and_layout():
    a = "int f(int x) {  // the value\n    return x + 1; /* one more */\n}\n"
    b = "int f(int x){return x+1;}"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only("return x + 2;") != bench._code_only("return x + 1;")


def test_stored_traffic_is_current_for_the_headline_kernel():
    """The stored HBM counters of the blocked sweep (the library's FP32 choice
    at 768^3) were taken on the code as it stands (else the benchmark reports
    traffic as null)."""
    with open(os.path.join(ROOT, "profiles", "traffic_counters.json")) as f:
        stored = json.load(f)
    entry = stored["sweep_blocked_p96_t8_largest_subdomain_768_fp32"]
    assert entry["sources_hash"] == bench.sources_hash("sweep_blocked")
    assert entry["bytes_per_launch"] >= entry["algorithmic_bytes_per_launch"]
    assert os.path.exists(os.path.join(ROOT, entry["summary"]))


def test_alu_roofline_of_the_blocked_sweep():
    """The blocked sweep reports the vector-ALU ceiling with the HBM rate
    beside it; slots per site update and the peak follow their definitions."""
    assert bench.ALU_SLOTS_PER_SITE == 46
    assert bench.ALU_PEAK_TSLOTS == pytest.approx(78.6432)
    V = 768 ** 3
    r = bench.roofline("sweep_blocked", V, 0.6, 3000.0, 2 * (V // 2) * 4, None, None)
    assert r["bound"] == "alu" and r["unit"] == "Tslot/s"
    assert r["achieved"] == pytest.approx(46 * V / 0.6e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert r["hbm"]["frac"] == pytest.approx(3000.0 / 8000.0)
    h = bench.roofline("halfsweep_stream", V, 0.35, 5000.0, 1, None, None)
    assert h["bound"] == "hbm" and h["frac"] == pytest.approx(5000.0 / 8000.0)


def test_time_to_1pct_scales_with_the_square_of_the_error():
    e = -2.0
    t = bench.time_to_1pct(10.0, 0.04, e)  # 2% after 10 s
    assert t["kind"] == "extrapolated"
    assert t["seconds"] == pytest.approx(40.0)
    assert t["eps_run"] == pytest.approx(0.02)
    assert bench.time_to_1pct(10.0, math.nan, e) is None
    assert bench.time_to_1pct(10.0, 0.04, 0.0) is None
    assert bench.time_to_1pct(10.0, 0.04, None) is None
