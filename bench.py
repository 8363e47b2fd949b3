"""Benchmark: PCG solves/s to 1e-6 relative residual with the DDLR preconditioner
on one MI355X, mixed precision (FP32 preconditioner inside FP64 CG) against the
FP64 preconditioner, with p50/p99 per-solve latency.

Workload (default): 7-point Laplacian on a 128^3 grid (n = 2,097,152), 4x4x4 box
subdomains (64 blocks), DDLR-1 with rank k = 32 from 64 Lanczos steps, 8
right-hand sides b = A x*, x* uniform[-1,1) with seeds 0..7, CG from x0 = 0 to
||r|| <= 1e-6 ||b||.  One step = one ddlr_solve of the 8-column batch; inputs
are resident in HBM before the timed region.

Prints one JSON line (see the keys below).  --gpus N with N > 1 exits: this
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def trsv_bytes(q: dict, nrhs: int, tbytes: int, nnz_b: int, rows_b: int) -> float:
    """Algorithmic HBM bytes of one launch of the per-block triangular-solve
    kernel: L and L^T of the B blocks (value + 4-byte column, once per launch),
    their row pointers, D^{-1}, and per right-hand side one read of x and one
    write of z over the B rows."""
    return 2.0 * nnz_b * (tbytes + 4) + 2.0 * 4 * rows_b + tbytes * rows_b + nrhs * 2.0 * tbytes * rows_b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--variant", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (see the design notes on sharding)"}))
        sys.exit(2)

    import torch

    import paper_1505_04341_amd as D
    import workloads as w

    cfg = w.config(args.config)
    A = cfg["A"]
    n, nrhs, k, m, p = A.n, cfg["nrhs"], cfg["k"], cfg["m"], cfg["p"]
    b, xs = w.rhs_from_solution(A, 0, nrhs)
    v0 = w.lanczos_start(n, 0)
    dev = "cuda:0"
    bt = torch.from_numpy(np.ascontiguousarray(b.T)).to(dev)
    xt = torch.zeros_like(bt)

    results = {}
    for name, prec in (("fp64", D.FP64), ("mixed", D.FP32)):
        log("setup", name)
        t0 = time.perf_counter()
        h = D.ddlr_setup(A, cfg["part"], p, k, args.variant, lanczos_steps=m, lanczos_start=v0, precision=prec)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        q = D.ddlr_query(h)
        log(name, "setup", f"{setup_s:.2f}s", "lanczos", f"{q['lanczos_ms']:.0f}ms", "theta", q["theta"])
        for _ in range(args.warmup):
            st, info = D.ddlr_solve(h, bt, xt)
        torch.cuda.synchronize()
        D.ddlr_profile(h, True)
        lat = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            st, info = D.ddlr_solve(h, bt, xt)  # synchronises the stream
            lat.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        prof = {c: D.ddlr_profile_read(h, c) for c in range(4)}
        D.ddlr_profile(h, False)
        its = [i["iters"] for i in info]
        rtrue = max(i["relres_true"] for i in info)
        log(name, "status", st, "iters", its, "max true relres", f"{rtrue:.2e}", "ms/step", 1e3 * total / args.steps)
        x = xt.cpu().numpy().T
        err = float(np.linalg.norm(x - xs) / np.linalg.norm(xs))
        results[name] = dict(h=h, q=q, setup_s=setup_s, total=total, lat=lat, prof=prof, its=its, status=st,
                             relres_true=rtrue, xerr=err, x=x)

    mixed, f64 = results["mixed"], results["fp64"]
    K = args.steps
    solves = K * nrhs
    value = solves / mixed["total"]
    lat_ms = np.array(mixed["lat"]) * 1e3
    # dominant kernel: the per-block triangular solve of the mixed path
    q = mixed["q"]
    part = cfg["part"]
    import paper_1505_04341_amd as D  # noqa: F811
    L, _ = D.ddlr_get_factor(mixed["h"])
    rows_b = int(q["m"])
    nnz_b = int(L.indptr[rows_b])
    tot_ms, launches = mixed["prof"][D.PROF_TRSV_BLOCKS]
    avg_s = tot_ms / max(launches, 1) / 1e3
    by = trsv_bytes(q, nrhs, 4, nnz_b, rows_b)
    achieved = by / avg_s / 1e9 if avg_s > 0 else 0.0
    kernel_share = {D.PROF_TRSV_BLOCKS: "trsv_blocks", D.PROF_TRSV_LEVELS: "trsv_levels", D.PROF_SPMV: "spmv",
                    D.PROF_LOWRANK: "lowrank"}
    breakdown = {kernel_share[c]: dict(ms_total=round(v[0], 3), launches=v[1],
                                       ms_per_step=round(v[0] / K, 3)) for c, v in mixed["prof"].items()}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(cfg, b, v0, args.variant)

    out = {
        "metric": "PCG solves/s to 1e-6 rel-res (mixed vs FP64 DDLR); p50/p99 solve latency",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * mixed["total"] / K, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 preconditioner / f64 CG",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: 7-point Laplacian 128^3, 4x4x4 boxes, DDLR-{args.variant} k={k}, "
                               f"{m} Lanczos steps, {nrhs} rhs per solve batch, CG to 1e-6",
                   "n": n, "nrhs": nrhs, "k": k, "p": p, "variant": args.variant},
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                       "p99": round(float(np.percentile(lat_ms, 99)), 3),
                       "note": "per solve; the 8 right-hand sides of a batch complete together"},
        "fp64": {"value": round(solves / f64["total"], 3), "ms_per_step": round(1e3 * f64["total"] / K, 3),
                 "p50_ms": round(float(np.percentile(np.array(f64["lat"]) * 1e3, 50)), 3),
                 "p99_ms": round(float(np.percentile(np.array(f64["lat"]) * 1e3, 99)), 3),
                 "iters": f64["its"], "max_relres_true": f64["relres_true"]},
        "mixed": {"iters": mixed["its"], "max_relres_true": mixed["relres_true"],
                  "x_rel_err_vs_xstar": mixed["xerr"],
                  "x_rel_diff_vs_fp64": float(np.linalg.norm(mixed["x"] - f64["x"]) / np.linalg.norm(f64["x"]))},
        "mixed_over_fp64": round(value / (solves / f64["total"]), 3),
        "setup_s": {"fp64": round(f64["setup_s"], 3), "mixed": round(mixed["setup_s"], 3)},
        "roofline": {"bound": "hbm", "kernel": "k_trsv_narrow<float>", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_launch": by, "avg_launch_us": round(avg_s * 1e6, 2)},
        "kernel_breakdown": breakdown,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(cfg, b, v0, variant):
    """The oracle (plain C, FP64, OpenMP over blocks/rows) on the host cores:
    full PCG solve of one right-hand side of the same workload."""
    try:
        from oracle import Oracle
    except Exception as e:  # pragma: no cover
        return {"error": str(e)}
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    log("cpu baseline: oracle setup")
    o = Oracle(cfg["A"], cfg["part"], cfg["p"])
    o.lowrank(variant, cfg["k"], cfg["m"], v0)
    t0 = time.perf_counter()
    x, info = o.pcg(b[:, :1])
    dt = time.perf_counter() - t0
    log("cpu baseline: its", info["its"][0], f"{dt:.1f}s")
    return {"value": round(1.0 / dt, 4), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"1 of the {b.shape[1]} right-hand sides (seed 0), full PCG solve to 1e-6 "
                      f"({int(info['its'][0])} iterations, {dt:.1f} s)"}


if __name__ == "__main__":
    main()
