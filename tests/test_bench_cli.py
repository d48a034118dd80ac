"""CPU checks of bench.py's contract pieces that need no GPU: it refuses more
than one GPU with a message, and it only reports recorded HBM traffic for
the kernel sources the counters were taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2202_09056_amd.profiling import kernel_source_hash  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_follows_the_kernel_sources():
    # a record taken on the current sources is reported, a stale one is not
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path) as f:
        data = json.load(f)
    assert data, "no traffic record"
    for key, ent in data.items():
        want = ent["bytes_per_launch"] if ent["source_hash"] == kernel_source_hash() else None
        assert bench.traffic_from_profiles(key) == want
        assert 0.5e9 < ent["bytes_per_launch"] < 0.7e9   # the 64^3 dominant kernel's scale
    assert bench.traffic_from_profiles("no such kernel") is None


def test_recorded_layouts_cover_the_bench_workload():
    # one line per operator of the 64^3 bench cube (rows cols blocks value_bytes C sorted)
    rec = os.path.join(ROOT, "profiles", "cube64_lognormal_tune_cache.txt")
    keys = {tuple(ln.split()[:4]) for ln in open(rec) if ln.strip()}
    assert ("274625", "274625", "7081535", "8") in keys      # A_1
    assert ("274625", "27668", "7650978", "8") in keys       # G_1 (the dominant kernel)
