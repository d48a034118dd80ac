"""Summaries of rocprofv3 CSV output for the solver's kernels.

    python -m paper_2202_09056_amd.profiling stats TRACE_DIR [--cmd CMD] > summary.md
    python -m paper_2202_09056_amd.profiling traffic FETCH_DIR WRITE_DIR COPY_FETCH_DIR \
        COPY_WRITE_DIR [--cmd CMD] [--json OUT.json --key KEY --kernel NAME --grid N]
    python -m paper_2202_09056_amd.profiling grids TRACE_DIR [--match REGEX] [--window KERNEL] [--min-pct P]

`stats` tabulates rocprofv3 --kernel-trace --stats output (kernel_stats.csv).
`grids` tabulates the same run's kernel_trace.csv per kernel and launch grid
(kernels whose name matches REGEX; with --window, only launches from 2 ms
before the first to 2 ms after the last launch of KERNEL in the last cluster
of its launches, i.e. the last solve that used it).
`traffic` turns two --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per
dispatch) into HBM bytes per launch, scaled by what the same counters read for
a plain 1 GiB device copy (bench.py --copy-calibration), and can record one
kernel's figure in a JSON file keyed by the current kernel sources.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 2 ** 30


# What a recorded HBM traffic figure of the dominant kernel depends on: the
# translation unit of the sliced-ELL kernels (k_sell), the host setup that
# fixes the operator's fill (hierarchy.cpp), the upload that fixes its
# layout, padding and row order (context.hip), and the recorded layouts the
# bench starts from.  The figure belongs to exactly these files.
KERNEL_SOURCES = ("paper_2202_09056_amd/csrc/device/kernels.hip", "paper_2202_09056_amd/csrc/device/kernels.hpp",
                  "paper_2202_09056_amd/csrc/device/launch.hpp", "paper_2202_09056_amd/csrc/device/context.hip",
                  "paper_2202_09056_amd/csrc/host/hierarchy.cpp", "profiles/cube64_lognormal_tune_cache.txt")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        path = os.path.join(ROOT, f)
        if os.path.exists(path):
            with open(path, "rb") as fh:
                h.update(fh.read())
        else:
            h.update(b"missing:" + f.encode())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = re.sub(r"\(.*", "", name)
    return name.replace("void saamg::", "").replace("saamg::", "").strip()


def _one(pattern: str) -> str:
    hits = glob.glob(pattern, recursive=True)
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def stats(trace_dir: str, cmd: str = "") -> str:
    path = _one(os.path.join(trace_dir, "**", "*kernel_stats.csv"))
    rows = list(csv.DictReader(open(path)))
    out = ["# Kernel time summary (rocprofv3 --kernel-trace --stats)", ""]
    if cmd:
        out += [f"Command: `{cmd}`", ""]
    out += ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def grids(trace_dir: str, match: str = "", window: str = "", min_pct: float = 0.0) -> str:
    path = _one(os.path.join(trace_dir, "**", "*kernel_trace.csv"))
    rows = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), _short(r["Kernel_Name"]), int(r["Grid_Size_X"]))
            for r in csv.DictReader(open(path))]
    rows.sort()
    if window:
        # the launches of `window` split into clusters at gaps of over 1 s;
        # keep the span of the last cluster, 2 ms either side
        ts = [r[0] for r in rows if r[2].startswith(window)]
        if not ts:
            raise SystemExit(f"no launch of {window}")
        first = len(ts) - 1
        while first > 0 and ts[first] - ts[first - 1] < 1_000_000_000:
            first -= 1
        lo, hi = ts[first] - 2_000_000, ts[-1] + 2_000_000
        rows = [r for r in rows if lo <= r[0] <= hi]
    pat = re.compile(match) if match else None
    agg = collections.defaultdict(list)
    for s, e, name, grid in rows:
        if pat is None or pat.search(name):
            agg[(name, grid)].append((e - s) / 1e3)
    total = sum(sum(v) for v in agg.values())
    out = ["| kernel | grid (threads) | launches | mean us | total ms | % |", "|---|---:|---:|---:|---:|---:|"]
    for (name, grid), v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        pct = 100.0 * sum(v) / total if total else 0.0
        if pct < min_pct:
            continue
        out.append(f"| `{name}` | {grid} | {len(v)} | {sum(v) / len(v):.1f} | {sum(v) / 1e3:.2f} | {pct:.1f} |")
    return "\n".join(out) + "\n"


def _counter(dirname: str):
    path = _one(os.path.join(dirname, "**", "*counter_collection.csv"))
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[(_short(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return agg


def _copy_factor(dirname: str) -> float:
    agg = _counter(dirname)
    vals = [v for (k, _), vs in agg.items() if "copyBuffer" in k for v in vs]
    kib = sorted(vals)[len(vals) // 2]
    return (COPY_BYTES / 1024.0) / kib


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir):
    ff, wf = _copy_factor(copy_fetch_dir), _copy_factor(copy_write_dir)
    fa, wa = _counter(fetch_dir), _counter(write_dir)
    rows = []
    for key in sorted(set(fa) & set(wa), key=lambda k: -sum(fa[k])):
        f = 1024.0 * ff * sum(fa[key]) / len(fa[key])
        w = 1024.0 * wf * sum(wa[key]) / len(wa[key])
        rows.append((key[0], key[1], len(fa[key]), f, w))
    return ff, wf, rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("stats")
    a.add_argument("trace_dir")
    a.add_argument("--cmd", default="")
    b = sub.add_parser("traffic")
    for n in ("fetch_dir", "write_dir", "copy_fetch_dir", "copy_write_dir"):
        b.add_argument(n)
    b.add_argument("--cmd", default="")
    b.add_argument("--json")
    b.add_argument("--key")
    b.add_argument("--kernel")
    b.add_argument("--grid", type=int)
    g = sub.add_parser("grids")
    g.add_argument("trace_dir")
    g.add_argument("--match", default="")
    g.add_argument("--window", default="")
    g.add_argument("--min-pct", type=float, default=0.0)
    args = ap.parse_args(argv)
    if args.what == "stats":
        sys.stdout.write(stats(args.trace_dir, args.cmd))
        return
    if args.what == "grids":
        sys.stdout.write(grids(args.trace_dir, args.match, args.window, args.min_pct))
        return
    ff, wf, rows = traffic(args.fetch_dir, args.write_dir, args.copy_fetch_dir, args.copy_write_dir)
    out = ["# HBM traffic per launch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)", ""]
    if args.cmd:
        out += [f"Command: `{args.cmd}`", ""]
    out += [f"Copy calibration (1 GiB read + 1 GiB written by a plain device copy): FETCH_SIZE "
            f"scale {ff:.4f}, WRITE_SIZE scale {wf:.4f}.", "",
            "| kernel | grid (threads) | launches | fetch MB | write MB |",
            "|---|---:|---:|---:|---:|"]
    for name, grid, n, f, w in rows[:40]:
        out.append(f"| `{name}` | {grid} | {n} | {f / 1e6:.2f} | {w / 1e6:.2f} |")
    sys.stdout.write("\n".join(out) + "\n")
    if args.json:
        hit = [r for r in rows if r[0] == args.kernel and (args.grid is None or r[1] == args.grid)]
        if not hit:
            raise SystemExit(f"kernel {args.kernel} (grid {args.grid}) not found")
        name, grid, n, f, w = hit[0]
        data = {}
        if os.path.exists(args.json):
            data = json.load(open(args.json))
        data[args.key] = {"bytes_per_launch": f + w, "fetch_bytes": f, "write_bytes": w,
                          "kernel": name, "grid": grid, "launches": n,
                          "source_hash": kernel_source_hash(), "command": args.cmd}
        with open(args.json, "w") as fh:
            json.dump(data, fh, indent=1)


if __name__ == "__main__":
    main()
