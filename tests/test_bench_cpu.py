"""bench.py's command-line contract that needs no GPU: one GPU only, and the
kernel name it reports for a launch shape is the one profilers show."""
import importlib.util
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused_with_a_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=300, cwd=ROOT)
    assert out.returncode != 0
    assert "one GPU" in out.stderr + out.stdout


def test_query_kernel_names():
    b = _bench_module()
    assert b.query_kernel_name(None) == "k_query_region<32, 2, 0>"
    assert b.query_kernel_name({"region": 64, "objs_per_lane": 1}) == "k_query_region<64, 1, 0>"
    assert b.query_kernel_name({"region": 32, "objs_per_lane": 0}) == "k_query_region<32, 1, 0>"
    assert b.query_kernel_name({"region": 0, "block": 8}) == "k_query<8>"
    assert b.query_kernel_name({"block": 0}) == "k_query<16>"
    assert b.query_kernel_name(None, aa=True) == "k_query_region<32, 2, 1>"
    assert b.query_kernel_name({"region": 0, "block": 16, "objs_per_lane": 2}, aa=True) == "k_query_region<32, 2, 1>"
    assert b.query_kernel_name({"region": 64, "objs_per_lane": 1}, aa=True) == "k_query_region<64, 1, 1>"
    assert b.fill_kernel_name(None) == "k_fill_region<32>"
    assert b.fill_kernel_name({"region": 64, "waves_per_wg": 4}) == "k_fill_region<64>"


def test_roofline_bound_is_the_slower_roof(tmp_path, monkeypatch):
    """The larger of bytes / 8 TB/s and flops / 78.6 TFLOP/s names the bound;
    the fraction is achieved over that roof's peak."""
    import json
    b = _bench_module()
    work = {"w-bytes": {"alg_bytes": 8_000_000_000, "alg_flops": 1_000_000},
            "w-flops": {"alg_bytes": 8_000_000, "alg_flops": 78_600_000_000}}
    f = tmp_path / "work.json"
    f.write_text(json.dumps(work))
    monkeypatch.setattr(b, "WORK_FILE", str(f))
    monkeypatch.setattr(b, "COUNTERS_GLOB", str(tmp_path / "none_*.json"))
    r = b.roofline_record("w-bytes", None, 0.1, 2000.0)      # 8 GB in 2 s: 4 GB/s
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["achieved"] - 4.0) < 1e-9 and abs(r["frac"] - 4.0 / 8000.0) < 1e-12
    assert abs(r["roofline_ms"] - 1.0) < 1e-12 and r["traffic"] is None
    r = b.roofline_record("w-flops", None, 0.1, 1000.0)      # 78.6 GFLOP in 1 s
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert abs(r["achieved"] - 0.0786) < 1e-12 and abs(r["frac"] - 0.001) < 1e-12
    assert list(r)[:6] == ["bound", "achieved", "peak", "unit", "frac", "traffic"]
    assert b.roofline_record("absent", None, 0.1, 1.0) is None


def test_roofline_from_extrapolated_counts(tmp_path, monkeypatch):
    """A workload counted on a per-zoom sample: requests at the covered zooms
    take the extrapolated figures, the others their mask bytes only, and the
    record says the figure is a lower bound."""
    import json
    b = _bench_module()
    work = {"w/zooms-3-4-extrapolated": {"alg_bytes": 1_000_000, "alg_flops": 78_600_000_000, "tiles": 3,
                                          "extrapolated": True, "per_zoom": {"3": {}, "4": {}}}}
    f = tmp_path / "work.json"
    f.write_text(json.dumps(work))
    monkeypatch.setattr(b, "WORK_FILE", str(f))
    monkeypatch.setattr(b, "COUNTERS_GLOB", str(tmp_path / "none_*.json"))
    r = b.roofline_record("w", None, 0.1, 1000.0, zooms=np.array([0, 3, 3, 4, 1]))
    assert r["alg_bytes_per_launch"] == 1_000_000 + 2 * 8192 and r["alg_flops_per_launch"] == 78_600_000_000
    assert r["bound"] == "alu" and abs(r["frac"] - 0.001) < 1e-12 and "lower bound" in r["alg_extrapolated"]
    assert b.roofline_record("w", None, 0.1, 1.0) is None          # zoom mix unknown
    with pytest.raises(AssertionError):
        b.roofline_record("w", None, 0.1, 1.0, zooms=np.array([3, 4]))   # another batch


def test_counters_are_matched_on_the_full_launch(tmp_path, monkeypatch):
    import json
    b = _bench_module()
    L = {"block": 0, "cand_cap": 128, "waves_per_wg": 1, "grid_wgs": 0, "region": 32, "objs_per_lane": 2,
         "cull_nodes": 0}
    run = {"workload": "w", "kernel": "k_query_region<32, 2, 0>", "launch": L,
           "query_source_sha256": b.source_hash(), "hbm_bytes_per_launch": 123.0}
    (tmp_path / "counters_query_w.json").write_text(json.dumps({"runs": [run]}))
    monkeypatch.setattr(b, "COUNTERS_GLOB", str(tmp_path / "counters_query_*.json"))
    assert b.committed_traffic("w", "k_query_region<32, 2, 0>", dict(L))[0] == 123.0
    assert b.committed_traffic("w", "k_query_region<32, 2, 0>", {**L, "cull_nodes": 32})[0] is None
    assert b.committed_traffic("w", "k_query_region<32, 2, 0>", None)[0] is None
    assert b.committed_traffic("v", "k_query_region<32, 2, 0>", dict(L))[0] is None
    run["query_source_sha256"] = "0" * 64
    (tmp_path / "counters_query_w.json").write_text(json.dumps(run))
    assert b.committed_traffic("w", "k_query_region<32, 2, 0>", dict(L))[0] is None
