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
    n, ldn = 19281, 19328
    w = bench.stage_work(s, "f32")
    assert w["similarity"] == ("flop", n * (n + 1) * 2048)  # unique entries of the symmetric S
    assert w["final"] == ("flop", 2 * 3368 * 15913 * n)     # 2.067e12
    # 34 candidates against 151 column blocks: the pruned selection reads the
    # block maxima and at least one block per candidate
    assert w["topk"] == ("byte", 4 * n * 151 + 4 * n * 34 * 128 + 8 * n * 34)
    # L = 1 with A* rows and the sum aggregator: the first layer is built from the
    # sparse rows and written once (no dense A*, no dense layer)
    assert w["propagate"] == ("byte", 4 * n * ldn + 13 * n * 26 + 4 * n)
    # the bf16x3 final product: the last layer writes two bf16 planes instead
    assert bench.stage_work(s, "f32", final="bf16x3")["propagate"][1] == 2 * 2 * n * ldn + 13 * n * 26 + 4 * n
    # max aggregator: dense A* rows, then one dense layer (rows read once, written once)
    wm = bench.stage_work(s, "f32", aggregator="max")
    assert wm["propagate"] == ("byte", 4 * n * ldn + 8 * n * 7 + 4 * n * ldn + 4 * n * 26)
    assert w["adjacency"] == ("byte", 14 * n * 26 + 16 * n)
    assert w["rescore"] == ("byte", n * 2048 * 4 + 8 * n * 34 + 8 * n * 26)
    assert bench.stage_work(s, "bf16")["topk"][1] == 2 * n * n + 8 * n * 42  # binary16 S
    assert bench.stage_work(s, "fp8", extra=16)["topk"][1] == 2 * n * n + 8 * n * 42
    assert bench.stage_work(s, "fp8")["topk"][1] == 2 * n * n + 8 * n * 58
    assert abs(w["final"][1] - 2.067e12) / 2.067e12 < 1e-3
    # FP32 rows of 2048 floats are read in place: no FP32 copy is written
    assert w["prep"] == ("byte", n * 2048 * 4 + 8 * n)
    assert bench.stage_work(s, "bf16")["prep"] == ("byte", n * 2048 * 4 + n * 2048 * 2 + 8 * n)


def test_stage_work_of_the_large_workload():
    s = synth.LARGE  # N = 50000, d = 512 (bf16 input), k1 = 20, k2 = 6, L = 2
    n, ldn = 50000, 50048
    w = bench.stage_work(s, "f32")
    # layer 1 kept as CSR rows, layer 2 written once as dense rows from them
    assert w["propagate"] == ("byte", 2 * 13 * n * 20 + 4 * n + 4 * n * ldn)
    assert w["prep"] == ("byte", n * 512 * 2 + n * 512 * 4 + 8 * n)
    # pruned selection at every precision (391 blocks per row)
    assert w["topk"] == ("byte", 4 * n * 391 + 4 * n * 28 * 128 + 8 * n * 28)
    assert bench.stage_work(s, "fp8")["topk"][1] == 4 * n * 391 + 2 * n * 52 * 128 + 8 * n * 52


# Stage times (ms) measured on one MI355X (bench.py's HIP events and the
# rocprofv3 kernel traces committed under profiles/).
MEASURED = {
    "mid_n19281_d2048": {"prep": 0.045, "similarity": 6.45, "topk": 0.128, "rescore": 0.27, "adjacency": 0.072,
                         "propagate": 0.245, "final": 15.2},
    "large_n50000_d512": {"prep": 0.0514, "similarity": 12.14, "topk": 0.29, "rescore": 0.27, "adjacency": 0.117,
                          "propagate": 2.78, "final": 283.4},
}


@pytest.mark.parametrize("spec", [synth.MID, synth.LARGE])
def test_no_roofline_fraction_above_one_at_measured_times(spec):
    # the work charged to a stage cannot have been done faster than the peak
    roof = bench.stage_rooflines(spec, MEASURED[spec.name])
    for stage, e in roof.items():
        assert e is None or 0 < e["frac"] <= 1.0, (stage, e)
    assert roof["final"]["bound"] == "mfma" and roof["topk"]["bound"] == "hbm"


def test_roofline_entries():
    # 2.067e12 flop in 15.2 ms -> 136 TFLOP/s of the FP32 peak
    e = bench.roofline_entry("final", "flop", 2.067e12, 15.2, "f32")
    assert e["bound"] == "mfma" and e["peak"] == 157.3 and e["unit"] == "TFLOP/s"
    assert e["achieved"] == pytest.approx(2.067e12 / 15.2e-3 / 1e12)
    assert e["frac"] == pytest.approx(e["achieved"] / 157.3)
    assert bench.roofline_entry("similarity", "flop", 1e12, 1.0, "bf16")["peak"] == 2500.0
    assert bench.roofline_entry("similarity", "flop", 1e12, 1.0, "fp8")["peak"] == 5000.0
    assert bench.roofline_entry("final", "flop", 1e12, 1.0, "bf16", "bf16")["peak"] == 2500.0
    assert bench.roofline_entry("final", "flop", 1e12, 1.0, "bf16", "bf16x3")["peak"] == pytest.approx(2500.0 / 3)
    h = bench.roofline_entry("topk", "byte", 1.487e9, 0.3, "f32")
    assert h["bound"] == "hbm" and h["unit"] == "GB/s" and h["frac"] == pytest.approx(1.487e9 / 0.3e-3 / 1e9 / 8000)
    assert bench.roofline_entry("final", "flop", 1.0, 0.0, "f32") is None


def test_cpu_baseline_entry_states_the_host():
    e = bench.cpu_baseline_entry(1e8, 2.0, "sample")
    assert e["value"] == pytest.approx(5e7) and e["kind"] == "oracle" and e["cores"] >= 1
    assert isinstance(e["cpu_model"], str) and e["cpu_model"]


def test_committed_traffic_matches_the_current_kernel_sources():
    # the summary under profiles/ records a hash of the dominant kernel's sources;
    # a stale summary would make bench.py report traffic as null
    t = bench.measured_traffic("mid_n19281_d2048", "f32", "final")
    assert t is not None and t["bytes"] > 0


def test_prep_bytes_charge_the_fp32_copy_only_when_it_is_made():
    # FP32 rows of a multiple of 64 floats are read in place; any other row
    # length (or bf16 input) is copied into the zero-padded FP32 layout
    n = 1000
    in_place = synth.ProblemSpec("p", 100, n - 100, 128, 10, 0.5)
    copied = synth.ProblemSpec("p", 100, n - 100, 130, 10, 0.5)
    bf16_in = synth.ProblemSpec("p", 100, n - 100, 128, 10, 0.5, dtype="bf16")
    assert bench.stage_work(in_place)["prep"] == ("byte", n * 128 * 4 + 8 * n)
    assert bench.stage_work(copied)["prep"] == ("byte", n * 130 * 4 + n * 192 * 4 + 8 * n)
    assert bench.stage_work(bf16_in)["prep"] == ("byte", n * 128 * 2 + n * 128 * 4 + 8 * n)
