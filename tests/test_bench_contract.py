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


@pytest.mark.parametrize("workload, stream", [("cylinder_full", 1), ("tension_cube100", 0), ("batch64", 1),
                                              ("confined150", 0)])
def test_traffic_summary_matches_the_kernel_name_the_benchmark_reads(workload, stream, monkeypatch):
    """The HBM-traffic summary holds the FP64 facet kernel under the name the
    benchmark looks up, with positive calibrated byte counts."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2603_13190_amd import rocprof_summary as RS
    path = os.path.join(ROOT, "profiles", f"facet_kernel_traffic_{workload}.json")
    with open(path) as f:
        rec = json.load(f)
    monkeypatch.setattr(RS, "source_sha1", lambda: rec["kernel_sources_sha1"])
    name = bench.facet_kernel_name("fp64", dict(tets_per_block=16, stream_facets=stream))
    assert name == f"k_facet<double, 1, 16, 0, {stream}>"
    t = bench.measured_traffic(workload, name)
    assert t is not None and t > 0
    cal = rec["calibration"]
    assert 1.9 < cal["fetch_scale"] < 2.1 and 0.9 < cal["write_scale"] < 1.1


def test_roofline_object_states_its_byte_basis():
    """The roofline object of the JSON line: fraction = layout bytes per
    launch / average launch time / 8 TB/s, with the survey's per-facet
    currency beside it."""
    sys.path.insert(0, ROOT)
    import bench
    r = {"facet_kernel_bytes": 1.6e9, "facet_kernel_avg_us": 400.0, "particle_kernel_avg_us": 50.0,
         "facet_kernel": "k_facet<double, 1, 16, 0, 1>", "facet_kernel_traffic": 1.65e9}
    ro = bench.roofline_of(r, 12_500_000, "fp64")
    assert ro["bound"] == "hbm" and ro["unit"] == "GB/s" and ro["peak"] == 8000.0
    assert abs(ro["achieved"] - 4000.0) < 1e-9 and abs(ro["frac"] - 0.5) < 1e-12
    assert abs(ro["alg_bytes_per_facet_update"] - 128.0) < 1e-9
    assert ro["traffic"] == 1.65e9 and "layout" in ro["byte_basis"]
    sc = ro["survey_currency"]
    assert sc["bytes_per_facet_update"] == 338.0
    assert abs(sc["equivalent_frac"] - 338.0 * 12.5e6 / 400e-6 / 1e9 / 8000.0) < 1e-12
