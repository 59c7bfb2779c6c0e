"""Benchmark: CPAA global PageRank on a Chung-Lu power-law graph on one MI355X.

Workload (default): Chung-Lu undirected graph, n = 4,000,000, target average
degree 16 (~64M stored entries), degree exponent 2.1, degrees in [1, 50000],
seed 2112001; damping c = 0.85; p = e/n; every solve certified to
||x - pi||_1 <= 1e-6 by the library's FP64 residual.  A step is one complete
solve (all terms of the series, the FP64 residual, any correction series and
the output), with p and x resident in HBM.

Prints one JSON line.  `value` is GTEPS = (stored entries x Chebyshev terms)
per second over the timed steps.  `roofline` covers the dominant kernel (the
fused term kernel): algorithmic bytes per launch over its average duration,
measured with HIP events on the solve's stream inside the library.
`cpu_baseline` times the FP64 oracle's CPAA on the host on a bounded sample of
the same workload (rank 0, N = 1 only).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS (nnz·terms/s) + PPR solves/s at ≤1e-6 L1, warm-start vs plain CPAA"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "term_w1_chung_lu_n4m_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2112_01743_amd", "csrc", "kernels_w1.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def term_bytes(n: int, nnz: int) -> int:
    """Algorithmic HBM bytes of one fused term launch (single right-hand side).

    col_idx 4*nnz + row_ptr 4*(n+1) + z_k gathered once 4n + z_{k-1} read 4n
    + z_{k+1} written 4n + FP64 accumulator read and written 16n.
    """
    return 4 * nnz + 4 * (n + 1) + 28 * n


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def load_traffic(n, nnz):
    """Measured HBM bytes per term launch from the committed counter runs, if they
    were taken on the current kernel source and the same workload."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash() or t.get("n") != n or t.get("nnz") != nnz:
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(g, c, seconds_target=15.0):
    """The FP64 oracle's CPAA (Alg. 1, scipy sparse products) on the same graph,
    for as many terms as fit in about `seconds_target` seconds."""
    import oracle
    b = (1.0 - c) * np.full(g.n, 1.0 / g.n)
    t0 = time.perf_counter()
    oracle.cpaa(g, b, c, 1)
    one = time.perf_counter() - t0
    terms = int(max(2, min(40, seconds_target / max(one / 2, 1e-3))))
    t0 = time.perf_counter()
    oracle.cpaa(g, b, c, terms)
    dt = time.perf_counter() - t0
    return {"value": g.nnz * terms / dt / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"FP64 oracle CPAA (scipy CSR products, single thread), first {terms} terms "
                      f"on the full benchmark graph, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=4_000_000)
    ap.add_argument("--avg-deg", type=float, default=16.0)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--nnz-per-thread", type=int, default=0)
    ap.add_argument("--xcd-remap", type=int, default=-1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters against a known byte count)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": src.numel() * 4,
                          "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design is described but not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import graphgen as gg
    from paper_2112_01743_amd import Plan

    c = 0.85
    t0 = time.perf_counter()
    g = gg.chung_lu(args.n, args.avg_deg, 2.1, seed=2112001, dmin=1.0, dmax=50000.0)
    log(f"graph n={g.n} nnz={g.nnz} maxdeg={int(np.diff(g.row_ptr).max())} "
        f"({time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    plan = Plan.from_graph(g, c, time_kernels=1, nnz_per_thread=args.nnz_per_thread,
                           xcd_remap=args.xcd_remap)
    info = plan.info()
    log(f"plan {info} ({time.perf_counter() - t0:.1f} s)")
    p = torch.full((g.n,), 1.0 / g.n, dtype=torch.float64, device="cuda")
    x = torch.empty_like(p)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        plan.solve(p, args.tol, out=x)
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, rep = plan.solve(p, args.tol, out=x)
        reps.append(rep)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if not all(r["certified"] for r in reps):
        log("WARNING: a timed solve was not certified")
    edges = sum(r["edges"] for r in reps)
    gteps = edges / wall / 1e9
    ms_terms = sum(r["ms_terms"] for r in reps)
    launches = sum(r["term_launches"] for r in reps)
    avg_launch_s = ms_terms / 1e3 / max(launches, 1)
    alg_bytes = term_bytes(g.n, g.nnz)
    achieved = alg_bytes / avg_launch_s / 1e9
    traffic = load_traffic(g.n, g.nnz)
    out = {
        "metric": METRIC,
        "value": gteps,
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 recurrence, f64 accumulation",
        "data": "synthetic",
        "config": {"workload": "chung_lu_global_pagerank", "n": g.n, "nnz": g.nnz,
                   "avg_degree_target": args.avg_deg, "gamma": 2.1, "max_degree_cap": 50000,
                   "seed": 2112001, "c": c, "tol_l1": args.tol, "personalization": "uniform",
                   "solves": args.steps},
        "solves_per_s": args.steps / wall,
        "terms": reps[-1]["terms"],
        "refine_terms": reps[-1]["refine_terms"],
        "cert_bound": reps[-1]["cert_bound"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "k_term_w1", "bytes_per_launch": alg_bytes,
                     "avg_launch_us": avg_launch_s * 1e6},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(g, c)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
