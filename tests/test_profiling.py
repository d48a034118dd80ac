"""CPU checks of the rocprofv3 summary helpers on a small synthetic trace."""
import csv
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2202_09056_amd import profiling  # noqa: E402

FIELDS = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X"]


def _trace(tmp_path, rows):
    d = tmp_path / "t"
    d.mkdir()
    with open(d / "x_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for name, s, e, g in rows:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": s, "End_Timestamp": e, "Grid_Size_X": g})
    return str(d)


def test_grids_groups_by_kernel_and_grid(tmp_path):
    ms = 1_000_000
    d = _trace(tmp_path, [("void saamg::k_a<float>(int)", 0, 10_000, 256),
                          ("void saamg::k_a<float>(int)", 20_000, 50_000, 256),
                          ("void saamg::k_a<float>(int)", 60_000, 64_000, 512),
                          ("saamg::k_b(double const*)", 70_000, 71_000, 64),
                          ("void saamg::k_a<float>(int)", 5_000 * ms, 5_000 * ms + 1_000, 256)])
    out = profiling.grids(d, match="k_a")
    lines = [ln for ln in out.splitlines() if ln.startswith("| `")]
    assert lines[0].startswith("| `k_a<float>` | 256 | 3 | 13.7 |")   # (10 + 30 + 1) us / 3
    assert lines[1].startswith("| `k_a<float>` | 512 | 1 | 4.0 |")
    assert "k_b" not in out
    # the window keeps the last cluster of k_a launches (the one 5 s later)
    out = profiling.grids(d, window="k_a")
    lines = [ln for ln in out.splitlines() if ln.startswith("| `")]
    assert len(lines) == 1 and lines[0].startswith("| `k_a<float>` | 256 | 1 | 1.0 |")
