"""Host-side contract of bench.py (no GPU): a multi-GPU request exits with a
message before any device work, and the memory-traffic figure is read from
the committed counter summary of the benchmarked mesh only."""
import importlib.util
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_traffic_is_read_per_mesh_size():
    bench = load_bench()
    assert bench.measured_traffic(12345) is None
    for n in (256, 2048):
        path = bench.TRAFFIC_SUMMARY.format(n=n)
        with open(path) as fh:
            d = json.loads(re.search(r"```json\n(.*?)\n```", fh.read(), re.S).group(1))
        assert f"{n}x{n}" in d["kernel"]
        # each figure is truncated to whole bytes on its own
        assert abs(d["traffic_bytes_per_launch"] - d["fetch_bytes"] - d["write_bytes"]) <= 1
        want = d["traffic_bytes_per_launch"] if d["kernel_source_sha256_16"] == \
            bench.kernel_source_hash() else None
        assert bench.measured_traffic(n) == want


def test_cpu_baseline_reports_cores_and_model():
    bench = load_bench()
    cb = bench.cpu_baseline(8, reps_all=1)
    assert cb["kind"] == "oracle" and cb["unit"] == "GDoF/s"
    assert 1 <= cb["cores"] <= len(os.sched_getaffinity(0))
    assert cb["value"] > 0 and cb["single_core"]["value"] > 0
    assert cb["single_core"]["cores"] == 1
    assert isinstance(cb["cpu_model"], str) and cb["cpu_model"]
    assert "8x8" in cb["sample"]
