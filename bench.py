#!/usr/bin/env python3
"""Benchmark of the band solve on one MI355X.

Metric: k-point band solves per second on the diamond-lattice workload
(conventional cubic cell, 8 spheres r = 0.13, eps 13 in 1, N = 64, i.e.
786,432 complex unknowns), 16 bands, relative residual 1e-8, 64 k-points along
Gamma-X-M-Gamma-R.  One step = one mfd_bands call over the whole k-path (warm
start from the previous k-point along the path, random start at the first).
A k-point counts when every band's residual, recomputed with the FP64
operator, is <= 1e-8.

Also reported (same JSON line):
  roofline      - the dominant kernel's achieved rate against its MI355X peak,
                  from HIP events recorded inside the library on the solve's
                  stream during the timed steps;
  stencil       - the same for the fused stencil (the metric's second part);
  cpu_baseline  - the FP64 CPU oracle timed on a bounded sample of the same
                  workload on this host.
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK = 8.0e12          # B/s
FP64_PEAK = 78.6e12        # FLOP/s, vector and matrix
FP32_PEAK = 157.3e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="diamond_n64")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--nk", type=int, default=0, help="k-points per step (0: the workload's path)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--guard", type=int, default=2)
    ap.add_argument("--streams", type=int, default=4, help="k-path segments solved concurrently")
    ap.add_argument("--roofline-nk", type=int, default=6, help="k-points of the single-stream timing pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--profile-only", action="store_true", help="one short step, no JSON (for rocprofv3)")
    ap.add_argument("--verbose", action="store_true", help="per-k statistics on stderr")
    return ap.parse_args()


def cpu_baseline(eps, L, k, m, iters, gpu_iters_per_k):
    """Time the FP64 oracle for a few LOBPCG iterations at one k-point of the
    same workload and scale by the GPU's iterations per k-point."""
    from oracle import lobpcg as olob
    from oracle import mfd as omfd
    from paper_2503_19379_amd import workloads
    N = eps.shape[0]
    n = 3 * N ** 3
    h = L / N
    mu = omfd.mu_from_eps(eps)
    g = omfd.gamma_rule(N, L, k)
    c = omfd.shift_rule(L, k)
    X0 = workloads.start_block(m, N, 0).reshape(m, n).T
    t0 = time.perf_counter()
    Pinv = np.linalg.inv(omfd.precond_matrices(N, L, k, g, 2, c))
    A = lambda X: omfd.apply_op(X.T.reshape(-1, 3, N, N, N), mu, k, h, g, 2, c).reshape(-1, n).T
    T = lambda R: omfd.precond_solve(R.T.reshape(-1, 3, N, N, N), N, L, k, g, 2, c, Pinv=Pinv).reshape(-1, n).T
    olob.lobpcg(A, T, X0, 1e-8, maxiter=iters)
    dt = time.perf_counter() - t0
    # lobpcg runs `iters` iterations plus the start-up and the final check
    per_iter = dt / (iters + 2)
    per_k = per_iter * gpu_iters_per_k
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / per_k, "unit": "k-points/s", "cores": cores, "kind": "oracle",
            "sample": f"{iters} oracle LOBPCG iterations (+ start-up and final check, {dt:.1f} s) at one "
                      f"k-point of the same workload, scaled to {gpu_iters_per_k:.1f} iterations per k-point "
                      f"(the GPU run's mean)"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path "
              "(k-points would shard across GPUs with no exchange; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2503_19379_amd import binding as B
    from paper_2503_19379_amd import workloads

    cfg = workloads.CONFIGS[args.workload]
    N, m = cfg["N"], cfg["nbands"]
    nk = args.nk or cfg["nk"]
    L = 1.0
    eps = workloads.crystal_eps(cfg["eps"], N)
    kpts = workloads.kpath(cfg["path"], cfg["nk"])[:nk]
    torch.cuda.set_device(0)
    ctx = B.mfd_build(N, L, 2, eps)
    opts = B.default_opts(precision=1 if args.precision == "mixed" else 0, warm_start=1, seed=0,
                          guard=args.guard, max_iter=500, streams=args.streams)

    def step():
        return B.mfd_bands(ctx, kpts, m, args.tol, opts)

    if args.profile_only:
        step()
        torch.cuda.synchronize()
        return
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(args.steps):
        results.append(step())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # Per-kernel durations: concurrent streams overlap kernels, so each
    # kernel's HIP-event time is taken in a separate single-stream pass over
    # the first k-points of the same path (same kernels, same shapes).
    B.mfd_profile(ctx, True)
    o1 = B.default_opts(precision=opts.precision, warm_start=1, seed=0, guard=args.guard, max_iter=500, streams=1)
    B.mfd_bands(ctx, kpts[:max(1, min(args.roofline_nk, nk))], m, args.tol, o1)
    torch.cuda.synchronize()
    prof = B.mfd_profile_read(ctx)
    B.mfd_profile(ctx, False)

    if args.verbose:
        for ev, st, status in results:
            for i, s in enumerate(st):
                print(f"k{i:3d} {np.array2string(kpts[i], precision=3)} iters={s['iters']:4d} "
                      f"res={s['max_rel_resid']:.2e} dbl={s['gamma_doublings']} spur={s['spurious']} "
                      f"ms={s['ms']:.1f} ev0={ev[i][0]:.6f} ev15={ev[i][-1]:.6f}", file=sys.stderr)
    ok = 0
    iters = []
    maxres = 0.0
    for ev, st, status in results:
        for s in st:
            iters.append(s["iters"])
            maxres = max(maxres, s["max_rel_resid"])
            if s["max_rel_resid"] <= args.tol and s["spurious"] == 0:
                ok += 1
    value = ok / dt
    n = 3 * N ** 3

    def rate(cat):
        p = prof[cat]
        if p["count"] == 0 or p["ms"] == 0:
            return None
        avg_s = p["ms"] / p["count"] * 1e-3
        return avg_s, p["bytes"] / p["count"]

    mb = m + args.guard
    rl = {}
    for cat in ("stencil", "precond", "gram", "update"):
        r = rate(cat)
        if r is None:
            continue
        avg_s, by = r
        if cat == "gram":
            flops = 8.0 * n * (3 * mb) * (6 * mb)
            rl[cat] = {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": FP64_PEAK / 1e12,
                       "unit": "TFLOP/s", "frac": flops / avg_s / FP64_PEAK, "traffic": None,
                       "avg_us": avg_s * 1e6, "total_ms": prof[cat]["ms"],
                       "per_launch": f"8 n (3mb)(6mb) = {flops:.3e} FLOP (full complex Gram, FP64 vector FMA)"}
        else:
            rl[cat] = {"bound": "hbm", "achieved": by / avg_s / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                       "frac": by / avg_s / HBM_PEAK, "traffic": None, "avg_us": avg_s * 1e6,
                       "total_ms": prof[cat]["ms"], "per_launch": f"{by:.4e} algorithmic bytes"}
    r = rate("rr")
    if r is not None:
        rl_rr = {"bound": "latency", "avg_us": r[0] * 1e6, "total_ms": prof["rr"]["ms"]}
    else:
        rl_rr = None
    dom = max(rl, key=lambda c: rl[c]["total_ms"]) if rl else None
    line = {
        "metric": "k-point band solves/sec at N=64, 16 bands, 1e-8 resid; stencil HBM GB/s vs peak",
        "value": value,
        "unit": "k-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: diamond cell, 8 spheres r=0.13a eps 13/1, N={N} "
                               f"({n} unknowns), {nk} k-points on {cfg['path']}, {m} bands, tol {args.tol:g}, "
                               f"{args.precision}",
                   "N": N, "nbands": m, "nk": nk, "tol": args.tol, "precision": args.precision,
                   "guard": args.guard, "streams": args.streams},
        "roofline_source": f"HIP events on the solve stream, single-stream pass over {min(args.roofline_nk, nk)} "
                           f"k-points of the same path after the timed steps",
        "roofline": dict(rl[dom], kernel=dom) if dom else None,
        "stencil": rl.get("stencil"),
        "kernels": dict(rl, rr=rl_rr) if rl_rr else rl,
        "iters_per_k": float(np.mean(iters)) if iters else None,
        "max_rel_resid": maxres,
        "converged_kpoints": ok,
        "total_kpoints": len(iters),
    }
    if not args.no_cpu_baseline:
        kidx = min(16, len(kpts) - 1)
        line["cpu_baseline"] = cpu_baseline(eps, L, kpts[kidx], m, args.cpu_iters,
                                            float(np.mean(iters)) if iters else 1.0)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
