"""bench.py's command-line contract that needs no GPU: one GPU only, and the
kernel name it reports for a launch shape is the one profilers show."""
import importlib.util
import os
import subprocess
import sys

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
    assert b.query_kernel_name(None) == "k_query_region<32, 2>"
    assert b.query_kernel_name({"region": 64, "objs_per_lane": 1}) == "k_query_region<64, 1>"
    assert b.query_kernel_name({"region": 32, "objs_per_lane": 0}) == "k_query_region<32, 1>"
    assert b.query_kernel_name({"region": 0, "block": 8}) == "k_query<8>"
    assert b.query_kernel_name({"block": 0}) == "k_query<16>"
