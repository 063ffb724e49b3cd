"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic work
it divides by, and the roofline entries it reports."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2012_07620_amd import synth  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line for a configuration it does not run


def test_stage_work_of_the_mid_workload():
    s = synth.MID  # Q = 3368, G = 15913, N = 19281, d = 2048, k1 = 26, k2 = 7, L = 1
    n = 19281
    w = bench.stage_work(s, "f32")
    assert w["similarity"] == ("flop", n * (n + 1) * 2048)  # unique entries of the symmetric S
    assert w["final"] == ("flop", 2 * 3368 * 15913 * n)     # 2.067e12
    assert w["topk"] == ("byte", 4 * n * n)                 # S read once, 1.487e9
    assert w["propagate"] == ("byte", 1 * (7 + 2) * 4 * n * n)
    assert w["rescore"] == ("flop", 2 * n * (26 + 8) * 2048)
    assert bench.stage_work(s, "bf16")["rescore"][1] == 2 * n * (26 + 16) * 2048
    assert bench.stage_work(s, "fp8")["rescore"][1] == 2 * n * (26 + 32) * 2048
    assert abs(w["final"][1] - 2.067e12) / 2.067e12 < 1e-3


def test_roofline_entries():
    # 2.067e12 flop in 15.2 ms -> 136 TFLOP/s of the FP32 peak
    e = bench.roofline_entry("final", "flop", 2.067e12, 15.2, "f32")
    assert e["bound"] == "mfma" and e["peak"] == 157.3 and e["unit"] == "TFLOP/s"
    assert e["achieved"] == pytest.approx(2.067e12 / 15.2e-3 / 1e12)
    assert e["frac"] == pytest.approx(e["achieved"] / 157.3)
    assert bench.roofline_entry("similarity", "flop", 1e12, 1.0, "bf16")["peak"] == 2500.0
    assert bench.roofline_entry("similarity", "flop", 1e12, 1.0, "fp8")["peak"] == 5000.0
    h = bench.roofline_entry("topk", "byte", 1.487e9, 0.3, "f32")
    assert h["bound"] == "hbm" and h["unit"] == "GB/s" and h["frac"] == pytest.approx(1.487e9 / 0.3e-3 / 1e9 / 8000)
    assert bench.roofline_entry("final", "flop", 1.0, 0.0, "f32") is None


def test_committed_traffic_matches_the_current_kernel_sources():
    # the summary under profiles/ records a hash of the dominant kernel's sources;
    # a stale summary would make bench.py report traffic as null
    t = bench.measured_traffic("mid_n19281_d2048", "f32", "final")
    assert t is not None and t["bytes"] > 0
