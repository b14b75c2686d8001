"""Host logic of the benchmark (no GPU): the one-GPU refusal, the recorded HBM
traffic tied to the kernel sources, and the roofline arithmetic."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_recorded_traffic_holds_for_the_current_sources_only(tmp_path):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    rec = json.load(open(path))
    for e in rec["entries"]:
        # every entry names its profile and was taken on the sources in the tree
        assert os.path.exists(os.path.join(ROOT, e["profile"]))
        got = bench.traffic_for(path, e["workload"], e["precision"])
        assert got == e["bytes_per_launch"]
        cal = e["calibration"]
        want = (e["fetch_kib_per_dispatch"] * cal["fetch_factor"]
                + e["write_kib_per_dispatch"] * cal["write_factor"]) * 1024
        assert abs(want - e["bytes_per_launch"]) <= 1.0
    # a record taken on other sources is not reported
    stale = dict(rec, entries=[dict(e, kernel_source_sha256_16="0" * 16) for e in rec["entries"]])
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(stale))
    assert bench.traffic_for(str(p), "twoboxes", "fp64") is None
    assert bench.traffic_for(str(tmp_path / "missing.json"), "twoboxes", "fp64") is None
    assert bench.traffic_for(path, "no such workload", "fp64") is None


def test_roofline_arithmetic():
    # 61.9M points of 12,288 flop in 33.3 ms: 22.8 TFLOP/s, 29% of the FP64 peak
    r = bench.roofline(33.3, 61_872_064, bench.PEAK_FP64_TFLOPS, 7.2e10, "k")
    assert r["achieved"] == pytest.approx(61_872_064 * 12_288 / 33.3e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6)
    assert 0.28 < r["frac"] < 0.30
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["traffic"] == 7.2e10
    # the trilinear element's contraction: (D B) 16 x 32 x 4 x 2 plus (B^T .) 32 x 32 x 4 x 2
    assert bench.FLOP_PER_POINT == 16 * 32 * 4 * 2 + 32 * 32 * 4 * 2
