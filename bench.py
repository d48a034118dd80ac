#!/usr/bin/env python3
"""Benchmark of the solve phase: CG preconditioned by one SA-AMG V-cycle over a
3x3-block hierarchy, FP64, on one MI355X.

Workload: 64^3 trilinear-brick unit cube (823,875 unknowns, 7,081,535 blocks),
E per element lognormal(0, 1) (seed 0), nu = 0.3, clamped at x = 0, body force
(0, 0, -1); hierarchy built once on the host (not timed).  One step = one
solve from x = 0 to an FP64 true relative residual <= 1e-8 with b and x
resident in HBM.  value = unknowns / (time per solve) = DoF/s.

Also reported: the roofline of the dominant kernel (level-1 smoothing sweep
fused with the r.z product, timed with HIP events on the solver's stream),
per-kernel timings, V-cycle bandwidth, and the CPU oracle timed on a sample of
the same workload recipe.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time-to-1e-8 residual & DoF/s; V-cycle HBM GB/s % peak "
          "(FP64 block vs FP32/learned)")
HBM_PEAK_GBS = 8000.0
OP_NAMES = {0: "spmv", 1: "restrict", 2: "prolong_add", 3: "jacobi0", 4: "smooth",
            5: "coarse_gemv", 6: "residual", 7: "smooth_dot", 8: "spmv_dot", 9: "vcycle",
            10: "cg_iteration"}
DOMINANT = (0, 7)  # (level, op): level-1 post-smoothing sweep fused with r.z


def kernel_source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2202_09056_amd", "csrc", "device")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_key):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE and
    WRITE_SIZE, scaled by a copy-kernel calibration), if recorded for the
    current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    ent = data.get(kernel_key)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(n_cube=40, repeats=2):
    """The oracle (scalar CSR, scipy) solve phase on a smaller cube of the same
    recipe, single-threaded; setup untimed."""
    from threadpoolctl import threadpool_limits
    import meshgen
    import oracle
    with threadpool_limits(1):
        p = meshgen.cube_lognormal(n_cube, seed=0)
        A = p.csr()
        h = oracle.build_hierarchy(A, p.coords)
        times, iters = [], 0
        for _ in range(repeats):
            t0 = time.perf_counter()
            r = oracle.amg_pcg(h, p.b, tol=1e-8)
            times.append(time.perf_counter() - t0)
            iters = r.iters
    t = sorted(times)[len(times) // 2]
    return {"value": p.n / t, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": (f"cube{n_cube}^3 lognormal (seed 0, {p.n} unknowns, same recipe as the "
                       f"workload), oracle scalar-CSR PCG + V-cycle to 1e-8, {iters} iterations, "
                       f"median of {repeats} solves of {sum(times):.1f} s total, setup untimed, "
                       f"1 thread")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=64, help="cube edge in elements")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timings", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (the solve of one problem "
              "on one MI355X); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import meshgen
    from paper_2202_09056_amd import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain copy kernel of known size: 1 GiB read + 1 GiB written per launch
        src = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": src.numel() * 8,
                                               "bytes_written": dst.numel() * 8, "launches": 5}}))
        return
    t_gen = time.perf_counter()
    p = meshgen.cube_lognormal(args.n, seed=0)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] workload cube{args.n} lognormal: n={p.n} nnzb={p.nnzb} "
          f"(generated in {t_gen:.1f} s)", file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        t_setup = time.perf_counter()
        solver = Solver(p.row_ptr, p.col, p.val, p.coords, stream=stream)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t_setup
        st = solver.stats()
        print(f"[bench] setup {t_setup:.2f} s (host {st.setup_ms / 1e3:.2f} s), levels "
              f"{[3 * st.nb[l] for l in range(st.levels)]}", file=sys.stderr, flush=True)
        b = torch.from_numpy(p.b).cuda()
        xs = [torch.zeros(p.n, dtype=torch.float64, device="cuda")
              for _ in range(args.warmup + args.steps)]
        torch.cuda.synchronize()
        for w in range(args.warmup):
            solver.solve(b, xs[w], tol=args.tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for k in range(args.steps):
            _, info, status = solver.solve(b, xs[args.warmup + k], tol=args.tol)
            infos.append((info.iters, info.rel_true_residual, info.solve_ms, status))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        print(f"[bench] timed {args.steps} solves", file=sys.stderr, flush=True)
        x = xs[-1]
        # independent FP64 check of the last solution on the host
        A = p.csr()
        xh = x.cpu().numpy()
        rel_host = float(np.linalg.norm(p.b - A @ xh) / np.linalg.norm(p.b))
        kernels = {}
        if not args.no_kernel_timings:
            for (lvl, op) in [(0, 6), (0, 7), (0, 8), (0, 1), (0, 2), (1, 6), (1, 4),
                              (1, 1), (1, 2), (0, 5), (0, 9), (0, 10)]:
                if op not in (5, 9, 10) and lvl + 1 >= st.levels:
                    continue
                ms, nbytes = solver.time_op(lvl, op, reps=20)
                kernels[f"L{lvl + 1}_{OP_NAMES[op]}"] = {
                    "ms": round(ms, 5), "bytes": nbytes, "GBps": round(nbytes / ms / 1e6, 1)}
        dom_ms, dom_bytes = solver.time_op(DOMINANT[0], DOMINANT[1], reps=50)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    iters = infos[-1][0]
    achieved = dom_bytes / dom_ms / 1e6
    vc = kernels.get("L1_vcycle")
    c1 = st.layout_A[0]
    dom_key = ("k_rowwave<double,double,MODE_SMOOTH_DOT>@L1" if c1 == 1 else
               f"k_sell<double,double,{abs(c1)},MODE_SMOOTH_DOT>@L1")
    traffic = traffic_from_profiles(dom_key)
    out = {
        "metric": METRIC,
        "value": p.n / (ms_per_step / 1e3),
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"cube{args.n}^3 Q1 elasticity, E lognormal(0,1) seed 0, nu 0.3, "
                         f"clamped x=0, body force; SA-AMG (eps 0.08, omega_p 2/3, 1+1 block "
                         f"Jacobi) + CG to rel. residual {args.tol:g}, FP64"),
            "unknowns": p.n,
            "blocks": p.nnzb,
            "levels": [3 * st.nb[l] for l in range(st.levels)],
            "operator_complexity": round(st.operator_complexity, 3),
            "iterations": iters,
            "time_to_tol_ms": ms_per_step,
            "ms_per_iteration": ms_per_step / max(iters, 1),
            "rel_true_residual_device": infos[-1][1],
            "rel_true_residual_host_check": rel_host,
            "host_setup_s": st.setup_ms / 1e3,
            "preconditioner_MB": st.device_bytes / 1e6,
        },
        "roofline": {
            "kernel": dom_key,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": dom_bytes,
            "ms_per_launch": dom_ms,
        },
        "vcycle": ({"ms": vc["ms"], "GBps": vc["GBps"], "frac_of_peak": round(vc["GBps"] / HBM_PEAK_GBS, 4)}
                   if vc else None),
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    solver.close()


if __name__ == "__main__":
    main()
