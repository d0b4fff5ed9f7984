"""Host-side checks of the benchmark script: the counter-traffic lookup is
keyed on the kernel sources and the grid size, and a request for more than
one GPU is refused."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_counter_traffic_follows_sources_and_size(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "roofline_counters.json")) as f:
        rec = json.load(f)["kernels"]
    recorded = rec["sweep_f64@128"]["source_sha256_16"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: recorded)
    for tag in bench.COUNTED:
        for n in (128, 256):
            r = rec[f"{tag}@{n}"]
            assert r["source_sha256_16"] == recorded      # one counter campaign per source state
            assert bench.counter_traffic(tag, n) == r["hbm_bytes"]
            # calibrated traffic is at least the algorithmic bytes (writes are exact)
            assert r["hbm_bytes"] >= r["algorithmic_bytes"] and r["cells"] == n ** 3
    assert bench.counter_traffic("sweep_f64", 96) is None          # no record at that size
    assert bench.counter_traffic("no_such_kernel", 128) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.counter_traffic("sweep_f64", 128) is None         # sources changed since


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
