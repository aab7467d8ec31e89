"""The benchmark's command-line contract and its link to the committed
counter summaries (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("workload", ["tension_cube100", "batch64"])
def test_traffic_summary_matches_the_kernel_name_the_benchmark_reads(workload, monkeypatch):
    """The HBM-traffic summary holds the FP64 facet kernel under the name the
    benchmark looks up, with positive calibrated byte counts."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2603_13190_amd import rocprof_summary as RS
    path = os.path.join(ROOT, "profiles", f"facet_kernel_traffic_{workload}.json")
    with open(path) as f:
        rec = json.load(f)
    monkeypatch.setattr(RS, "source_sha1", lambda: rec["kernel_sources_sha1"])
    t = bench.measured_traffic(workload, "k_facet<double, 1, 16, 0>")
    assert t is not None and t > 0
    cal = rec["calibration"]
    assert 1.9 < cal["fetch_scale"] < 2.1 and 0.9 < cal["write_scale"] < 1.1
