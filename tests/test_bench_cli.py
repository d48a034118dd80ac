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


def test_solve_times_are_named_after_the_criterion_met():
    class Info:
        def __init__(self, converged):
            self.converged = converged
    assert bench._time_fields(1.234, 0, Info(1)) == {"time_to_1e-8_ms": 1.23, "time_ms": 1.23}
    assert bench._time_fields(2.0, 0, Info(2)) == {"time_to_recurrence_1e-8_ms": 2.0, "time_ms": 2.0}
    # a stop short of the target (status 1, not converged) never reports a time to 1e-8
    assert bench._time_fields(3.0, 1, Info(0)) == {"time_ms_not_converged": 3.0, "time_ms": 3.0}
    assert "time_to_1e-8_ms" not in bench._time_fields(3.0, -6, Info(1))
