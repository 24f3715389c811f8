#!/usr/bin/env python3
"""Benchmark of the band solve on one MI355X.

Metric: k-point band solves per second on the diamond-lattice workload
(conventional cubic cell, 8 spheres r = 0.13, eps 13 in 1, N = 64, i.e.
786,432 complex unknowns), 16 bands, relative residual 1e-8, 64 k-points along
Gamma-X-M-Gamma-R, in mixed precision (FP32 corrections, FP64 refinement).
One step = one mfd_bands call over the whole k-path, cut into concurrently
solved segments (random start at a segment's first k-point, warm start from
the previous k-point after it).  A k-point counts when every band's residual,
recomputed with the FP64 operator, is <= 1e-8.

Also reported (same JSON line):
  variants      - one timed step each of the plain FP64 solve, of the
                  learned warm start, of a 32-crystal batch and of the band
                  structure and band-gap ratio of the curved-interface cubic
                  cell (N = 120), on the same GPU;
  roofline      - the dominant kernel's achieved rate against its MI355X peak,
                  from HIP events recorded inside the library on the solve's
                  stream during the timed steps;
  stencil       - the metric's second part: the fused stencil alone on a
                  full 16-band FP32 block (HIP events over back-to-back
                  calls), with the FP64-arithmetic form and the solver's own
                  launches beside it;
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
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"],
                    help="mixed: FP32 corrections with FP64 refinement, the workload's own precision")
    ap.add_argument("--nk", type=int, default=0, help="k-points per step (0: the workload's path)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--guard", type=int, default=2)
    ap.add_argument("--streams", type=int, default=12, help="k-path segments solved concurrently")
    ap.add_argument("--warm", default="prev", choices=["prev", "learned"],
                    help="start block after a segment's first k-point: previous k, or the learned proposal")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the one-step comparison runs (FP64 solve, learned warm start)")
    ap.add_argument("--roofline-nk", type=int, default=6, help="k-points of the single-stream timing pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--profile-only", action="store_true", help="one short step, no JSON (for rocprofv3)")
    ap.add_argument("--stencil-only", action="store_true",
                    help="only the full-block stencil timing (for rocprofv3); prints its JSON object")
    ap.add_argument("--lattice-only", action="store_true",
                    help="only the general-lattice operator timing on the BCC gyroid at N = 120 (for rocprofv3); "
                         "prints its JSON object")
    ap.add_argument("--copy-calib", action="store_true",
                    help="with --profile-only, --stencil-only or --lattice-only: also run a plain 1 GiB read + 1 GiB write copy, "
                         "the reference for scaling the HBM byte counters")
    ap.add_argument("--verbose", action="store_true", help="per-k statistics on stderr")
    return ap.parse_args()


COPY_BYTES = 1 << 30
PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
KERNEL_SOURCES = {"update": "gemm.hip", "gram": "gemm.hip", "stencil": "stencil.hip", "precond": "fft.hip"}


def measured_traffic(workload, precision):
    """HBM bytes per launch from the committed rocprofv3 counter summaries
    (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size), or None
    for a kernel whose source changed since the counters were taken."""
    import hashlib
    out = {}
    for cat, src in KERNEL_SOURCES.items():
        path = os.path.join(PROFILES, f"{cat}_{workload}_{precision}_hbm_traffic.md")
        if not os.path.exists(path):
            continue
        fields = {}
        with open(path) as f:
            for line in f:
                if ":" in line and line.startswith("- "):
                    key, _, val = line[2:].partition(":")
                    fields[key.strip()] = val.strip().strip("`")
        src_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2503_19379_amd", "csrc", src)
        with open(src_path, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
        if fields.get("source_sha256") == digest and "traffic_bytes_per_launch" in fields:
            out[cat] = float(fields["traffic_bytes_per_launch"])
    return out


def batch_workers(args):
    return min(2 * args.streams, 16)


def batch_variant(B, args, torch, count):
    """Many crystals of uneven grids in one mfd_bands_batch call: 32 seeded
    random-field crystals (N = 24, 32, 48, 64 in turn), 8 k-points on
    Gamma-X-M-Gamma-R and 12 bands each, mixed precision, crystals handed to
    the workers in a queue.  One timed call after an untimed one that sizes
    every crystal's workspace."""
    from paper_2503_19379_amd import workloads
    cfg = workloads.CONFIGS["random_batch"]
    crystals = workloads.random_batch_crystals(cfg["ncrys"], cfg["Ns"])
    ctxs = [B.mfd_build(N, 1.0, 2, eps) for N, eps in crystals]
    kp = workloads.kpath(cfg["path"], cfg["nk"])
    o = B.default_opts(precision=1, warm_start=1, seed=0, guard=args.guard, max_iter=500,
                       streams=batch_workers(args))
    B.mfd_bands_batch(ctxs, [kp[:1]] * len(ctxs), cfg["nbands"], cfg["tol"], o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs, sts, status = B.mfd_bands_batch(ctxs, [kp] * len(ctxs), cfg["nbands"], cfg["tol"], o)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok, iters, maxres = count([(None, st, status) for st in sts])
    for c in ctxs:
        c.close()
    return {"value": ok / dt, "unit": "k-points/s", "steps": 1, "ms_per_step": dt * 1e3,
            "iters_per_k": float(np.mean(iters)), "converged_kpoints": ok, "total_kpoints": len(iters),
            "max_rel_resid": maxres, "precision": "mixed", "warm_start": "prev", "workers": o.streams,
            "workload": f"{cfg['ncrys']} random-field crystals (correlation length 0.15, 30% eps 13 in 1), "
                        f"N in {cfg['Ns']}, {cfg['nk']} k-points on {cfg['path']}, {cfg['nbands']} bands, "
                        f"tol {cfg['tol']:g}"}


def band_gap_variant(B, args, torch):
    """Section 6.2's curved-interface cubic cell (sphere 0.345 + three
    cylinders 0.11, eps 13 in 1, M_0 set per edge) at N = 120: 10 bands along
    Gamma-X-M-Gamma-R-X-M-R with every symmetry point, the paper's tolerance
    1e-5, mixed precision, then the band-gap ratio.  One timed call after an
    untimed one at the first k-point."""
    from paper_2503_19379_amd import workloads
    cfg = workloads.CONFIGS["sc_sphere_cyl"]
    N = cfg["N"]
    kp = workloads.kpath_vertices(cfg["path"], cfg["nk"])
    ctx = B.mfd_build_mu(N, 1.0, 2, workloads.mu_sc_sphere_cylinders(N))
    o = B.default_opts(precision=1, warm_start=1, seed=0, guard=2, max_iter=500, streams=args.streams)
    B.mfd_bands(ctx, kp[:1], cfg["nbands"], cfg["tol"], o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, st, status = B.mfd_bands(ctx, kp, cfg["nbands"], cfg["tol"], o)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ratio, below = B.mfd_gap_ratio(ev, kp)
    ctx.close()
    ok = sum(1 for x in st if x["max_rel_resid"] <= cfg["tol"])
    return {"value": ok / dt, "unit": "k-points/s", "steps": 1, "ms_per_step": dt * 1e3,
            "iters_per_k": float(np.mean([x["iters"] for x in st])), "converged_kpoints": ok,
            "total_kpoints": len(st), "gap_ratio": ratio, "gap_above_band": below,
            "gap_ratio_paper": cfg["gap_ratio_paper"], "N_paper": cfg["N_paper"],
            "workload": f"simple cubic sphere r 0.345 + 3 cylinders r 0.11, eps 13 in 1, M_0 per edge, N = {N}, "
                        f"{len(kp)} k-points on {cfg['path']}, {cfg['nbands']} bands, tol {cfg['tol']:g}, mixed"}


def lattice_op_direct(B, ctx, k, m, N, torch, reps=20):
    """The general-lattice operator alone (the fused z-marching kernel at
    order 2) on a block of m FP32-stored bands, FP64 arithmetic as the mixed
    solve applies it: mean duration of `reps` back-to-back mfd_op_apply calls
    between HIP events on their stream.  Algorithmic bytes per call: X read
    and Y written once (2 x 24 B per cell and band) plus mu (24 B per cell)
    once; the halo ring and neighbour planes come from LDS."""
    n3 = N ** 3
    g = torch.Generator(device="cuda").manual_seed(0)
    X = torch.randn((m, 3, N, N, N), dtype=torch.complex64, device="cuda", generator=g)
    Y = torch.empty_like(X)
    s = torch.cuda.Stream()
    for _ in range(3):
        B.mfd_op_apply(ctx, k, X, Y, stream=s.cuda_stream, fp64_arith=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        B.mfd_op_apply(ctx, k, X, Y, stream=s.cuda_stream, fp64_arith=True)
    e1.record(s)
    e1.synchronize()
    avg_s = e0.elapsed_time(e1) * 1e-3 / reps
    by = 48.0 * n3 * m + 24.0 * n3
    del X, Y
    torch.cuda.synchronize()
    return {"achieved": by / avg_s / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": by / avg_s / HBM_PEAK,
            "avg_us": avg_s * 1e6, "bytes_per_call": by, "nbands": m, "N": N, "calls": reps,
            "form": "FP32 storage, FP64 arithmetic, one z-marching pass (lattice_fused_kernel)"}


def lattice_only(B, torch):
    """The BCC gyroid context at N = 120 and the lattice operator timing
    alone (for rocprofv3)."""
    from paper_2503_19379_amd import workloads
    cfg = workloads.CONFIGS["bcc_gyroid"]
    N = cfg["Ns"][-1]
    ctx = B.mfd_build_lattice_mu(N, workloads.lattice_vectors("bcc"), 2, workloads.mu_bcc_gyroid(N))
    out = lattice_op_direct(B, ctx, np.array(cfg["k"]), cfg["nbands"] + 2, N, torch)
    ctx.close()
    return out


def gyroid_variant(B, args, torch):
    """Section 6.3's BCC single gyroid (eps 16 in 1, M_0 per edge, general
    lattice operator).  (1) Table time_comp_bc's workload: the first 10
    bands at k = (pi, pi, pi)/l to the paper's tolerance 1e-5 from a random
    start, N = 100 and 120, one timed solve after an untimed one; the paper's
    steps and its A100 seconds are carried beside for context.  (2) The band
    structure on H'-Gamma-P-N-H at N = 120 and its gap ratio.  (3) The
    lattice operator alone on a 12-band block at N = 120
    (lattice_op_direct)."""
    from paper_2503_19379_amd import workloads
    cfg = workloads.CONFIGS["bcc_gyroid"]
    A = workloads.lattice_vectors("bcc")
    kP = np.array([cfg["k"]])
    out = {"workload": "BCC single gyroid g > 1.1, eps 16 in 1, M_0 per edge, general-lattice operator, "
                       f"{cfg['nbands']} bands, tol {cfg['tol']:g}, mixed precision"}
    for N in cfg["Ns"]:
        ctx = B.mfd_build_lattice_mu(N, A, 2, workloads.mu_bcc_gyroid(N))
        o = B.default_opts(precision=1, warm_start=0, seed=0, guard=2, max_iter=500, streams=1)
        B.mfd_bands(ctx, kP, cfg["nbands"], cfg["tol"], o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, st, status = B.mfd_bands(ctx, kP, cfg["nbands"], cfg["tol"], o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"P_N{N}"] = {"value": 1.0 / dt, "unit": "k-points/s", "ms": dt * 1e3, "iters": st[0]["iters"],
                          "max_rel_resid": st[0]["max_rel_resid"], "status": status,
                          "paper_steps": cfg["steps_paper"][N], "paper_a100_s": cfg["gpu_s_paper"][N]}
        if N == cfg["Ns"][-1]:
            kp = workloads.kpath_vertices(cfg["path"], cfg["nk"], points=workloads.bcc_points())
            o = B.default_opts(precision=1, warm_start=1, seed=0, guard=2, max_iter=500, streams=args.streams)
            t0 = time.perf_counter()
            ev, st, status = B.mfd_bands(ctx, kp, cfg["nbands"], cfg["tol"], o)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ratio, below = B.mfd_gap_ratio(ev, kp)
            ok = sum(1 for x in st if x["max_rel_resid"] <= cfg["tol"])
            out[f"path_N{N}"] = {"value": ok / dt, "unit": "k-points/s", "ms": dt * 1e3, "kpoints": len(kp),
                                 "converged_kpoints": ok, "gap_ratio": ratio, "gap_above_band": below,
                                 "gap_ratio_paper": cfg["gap_ratio_paper"], "N_paper": cfg["N_paper"]}
            out["lattice_operator"] = lattice_op_direct(B, ctx, kP[0], cfg["nbands"] + 2, N, torch)
        ctx.close()
    return out


def fcc_gap_variant(B, args, torch):
    """Section 6.3's FCC sp3 diamond (spheres and bond spheroids, eps 13 in
    1, M_0 per edge) at N = 100: 10 bands on X-U-L-Gamma-X-W-K with every
    symmetry point, tol 1e-5, mixed precision, one timed call, then the
    band-gap ratio."""
    from paper_2503_19379_amd import workloads
    cfg = workloads.CONFIGS["fcc_diamond"]
    N = 100
    kp = workloads.kpath_vertices(cfg["path"], cfg["nk"], points=workloads.fcc_points())
    ctx = B.mfd_build_lattice_mu(N, workloads.lattice_vectors("fcc"), 2, workloads.mu_fcc_diamond(N))
    o = B.default_opts(precision=1, warm_start=1, seed=0, guard=2, max_iter=500, streams=args.streams)
    B.mfd_bands(ctx, kp[:1], cfg["nbands"], cfg["tol"], o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, st, status = B.mfd_bands(ctx, kp, cfg["nbands"], cfg["tol"], o)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ratio, below = B.mfd_gap_ratio(ev, kp)
    ctx.close()
    ok = sum(1 for x in st if x["max_rel_resid"] <= cfg["tol"])
    return {"value": ok / dt, "unit": "k-points/s", "ms": dt * 1e3, "kpoints": len(kp), "converged_kpoints": ok,
            "iters_per_k": float(np.mean([x["iters"] for x in st])), "gap_ratio": ratio, "gap_above_band": below,
            "gap_ratio_paper": cfg["gap_ratio_paper"], "N_paper": cfg["N_paper"],
            "workload": f"FCC sp3 diamond, spheres r 0.12 + bond spheroids of minor radius 0.11, eps 13 in 1, "
                        f"M_0 per edge, N = {N}, {len(kp)} k-points on {cfg['path']}, {cfg['nbands']} bands, "
                        f"tol {cfg['tol']:g}, mixed"}


def stencil_object(direct, timed, single):
    out = dict(direct["fp32"], form="fp32 storage and arithmetic, full 16-band block, 30 back-to-back calls")
    out["fp32_storage_fp64_arith"] = direct["fp32_storage_fp64_arith"]
    if timed is not None:
        out["in_solve"] = {
            "timed_region": {k: timed[k] for k in ("achieved", "frac", "avg_us", "launches", "traffic")},
            "single_stream": {k: single[k] for k in ("achieved", "frac", "avg_us")} if single else None,
            "note": "soft-locked launches (about 10 active bands) in FP64 arithmetic; the timed region's "
                    "durations include the wait for CUs held by the concurrent segments"}
    return out


def stencil_direct(B, ctx, k, m, N, torch, reps=30):
    """The fused stencil alone on a full block of m bands (no soft locking),
    with nothing else on the chip: mean duration of `reps` back-to-back
    mfd_op_apply calls between HIP events on the stream they launch on.
    Algorithmic bytes per call: X read and Y written once (2 x 24 N^3 m bytes
    of complex64) plus mu on the 3 N^3 edges once (FP32 copy: 12 N^3 bytes;
    FP64: 24 N^3), the halos coming from LDS or cache."""
    n3 = N ** 3
    g = torch.Generator(device="cuda").manual_seed(0)
    X = torch.randn((m, 3, N, N, N), dtype=torch.complex64, device="cuda", generator=g)
    Y = torch.empty_like(X)
    s = torch.cuda.Stream()
    out = {}
    for name, f64, mu_bytes in (("fp32", False, 12), ("fp32_storage_fp64_arith", True, 24)):
        for _ in range(3):
            B.mfd_op_apply(ctx, k, X, Y, stream=s.cuda_stream, fp64_arith=f64)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            B.mfd_op_apply(ctx, k, X, Y, stream=s.cuda_stream, fp64_arith=f64)
        e1.record(s)
        e1.synchronize()
        avg_s = e0.elapsed_time(e1) * 1e-3 / reps
        by = 48.0 * n3 * m + mu_bytes * n3
        out[name] = {"achieved": by / avg_s / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": by / avg_s / HBM_PEAK, "avg_us": avg_s * 1e6, "bytes_per_call": by,
                     "nbands": m, "calls": reps}
    del X, Y
    torch.cuda.synchronize()
    return out


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
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except ImportError:
        cores = 1
    return {"value": 1.0 / per_k, "unit": "k-points/s", "cores": cores, "kind": "oracle",
            "sample": f"{iters} oracle LOBPCG iterations (+ start-up and final check, {dt:.1f} s) at one "
                      f"k-point of the same workload, scaled to {gpu_iters_per_k:.1f} iterations per k-point "
                      f"(the GPU run's mean)"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path "
              "(k-points would shard across GPUs with no exchange between them)", file=sys.stderr)
        sys.exit(2)
    # One hardware queue per concurrent k-path segment: with fewer, segments
    # share a queue and one segment's one-workgroup Rayleigh-Ritz step holds up
    # the other's kernels.  HIP reads this when it initialises, below.
    # The batch variant's crystals run on twice as many workers (their small
    # solves are bound by the host round trip of each iteration).
    queues = max(args.streams, 0 if args.no_variants else batch_workers(args))
    if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < queues:
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(queues, 32))
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
    def make_opts(precision, warm):
        return B.default_opts(precision=1 if precision == "mixed" else 0, warm_start=2 if warm == "learned" else 1,
                              seed=0, guard=args.guard, max_iter=500, streams=args.streams)

    opts = make_opts(args.precision, args.warm)

    def step(o=opts):
        return B.mfd_bands(ctx, kpts, m, args.tol, o)

    def count(results):
        ok, iters, maxres = 0, [], 0.0
        for ev, st, status in results:
            for s in st:
                iters.append(s["iters"])
                maxres = max(maxres, s["max_rel_resid"])
                if s["max_rel_resid"] <= args.tol and s["spurious"] == 0:
                    ok += 1
        return ok, iters, maxres

    def copy_calibration():
        x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()

    if args.lattice_only:
        print(json.dumps(lattice_only(B, torch)))
        if args.copy_calib:
            copy_calibration()
        return
    if args.stencil_only:
        print(json.dumps(stencil_direct(B, ctx, kpts[min(16, nk - 1)], m, N, torch)))
        if args.copy_calib:
            copy_calibration()
        return
    if args.profile_only:
        step()
        torch.cuda.synchronize()
        if args.copy_calib:
            copy_calibration()
        return
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # Per-kernel durations: HIP events recorded by the library around each
    # launch on the stream it is launched on, during the timed steps.
    B.mfd_profile(ctx, True)
    t0 = time.perf_counter()
    results = []
    for _ in range(args.steps):
        results.append(step())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = B.mfd_profile_read(ctx)
    # The same kernels without the overlap of concurrent segments: a
    # single-stream pass over the first k-points of the path.
    B.mfd_profile(ctx, True)
    o1 = B.default_opts(precision=opts.precision, warm_start=1, seed=0, guard=args.guard, max_iter=500, streams=1)
    B.mfd_bands(ctx, kpts[:max(1, min(args.roofline_nk, nk))], m, args.tol, o1)
    torch.cuda.synchronize()
    prof_iso = B.mfd_profile_read(ctx)
    B.mfd_profile(ctx, False)

    if args.verbose:
        for ev, st, status in results:
            for i, s in enumerate(st):
                print(f"k{i:3d} {np.array2string(kpts[i], precision=3)} iters={s['iters']:4d} "
                      f"res={s['max_rel_resid']:.2e} dbl={s['gamma_doublings']} spur={s['spurious']} "
                      f"ms={s['ms']:.1f} ev0={ev[i][0]:.6f} ev15={ev[i][-1]:.6f}", file=sys.stderr)
    ok, iters, maxres = count(results)
    value = ok / dt

    # One-step comparison runs on the same GPU: the plain FP64 solve, and the
    # learned warm start (each after an untimed call that sizes its workspaces).
    variants = {}
    if not args.no_variants:
        for name, prec, warm in (("fp64_prev", "fp64", "prev"), ("mixed_learned", "mixed", "learned")):
            if (prec, warm) == (args.precision, args.warm):
                continue
            o = make_opts(prec, warm)
            B.mfd_bands(ctx, kpts[:min(nk, args.streams)], m, args.tol, o)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = step(o)
            torch.cuda.synchronize()
            d1 = time.perf_counter() - t1
            vok, vit, vres = count([r])
            variants[name] = {"value": vok / d1, "unit": "k-points/s", "steps": 1, "ms_per_step": d1 * 1e3,
                              "iters_per_k": float(np.mean(vit)), "converged_kpoints": vok,
                              "max_rel_resid": vres, "precision": prec, "warm_start": warm}
        variants["random_batch"] = batch_variant(B, args, torch, count)
        variants["sc_sphere_cyl_gap"] = band_gap_variant(B, args, torch)
        variants["bcc_gyroid"] = gyroid_variant(B, args, torch)
        variants["fcc_diamond_gap"] = fcc_gap_variant(B, args, torch)
    n = 3 * N ** 3

    mb = m + args.guard
    traffic = measured_traffic(args.workload, args.precision)

    def rooflines(prof):
        rl = {}
        for cat in ("stencil", "precond", "gram", "update", "rr"):
            p = prof[cat]
            if p["count"] == 0 or p["ms"] == 0:
                continue
            avg_s = p["ms"] / p["count"] * 1e-3
            by = p["bytes"] / p["count"]
            if cat == "rr":
                rl[cat] = {"bound": "latency", "avg_us": avg_s * 1e6, "total_ms": p["ms"], "launches": p["count"]}
            elif cat == "gram":
                # the library records 8 n K (K+1) per launch for its basis of K
                # columns (soft locking shrinks K): two Hermitian products, upper halves
                flops = by
                rl[cat] = {"bound": "mfma", "achieved": flops / avg_s / 1e12, "peak": FP64_PEAK / 1e12,
                           "unit": "TFLOP/s", "frac": flops / avg_s / FP64_PEAK, "traffic": traffic.get(cat),
                           "avg_us": avg_s * 1e6, "total_ms": p["ms"], "launches": p["count"],
                           "per_launch": f"S^H S and S^H AS, Hermitian: 8 n K (K+1) = {flops:.3e} FLOP "
                                         f"(mean over launches; K = mb + 2 na with na active bands)"}
            else:
                rl[cat] = {"bound": "hbm", "achieved": by / avg_s / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                           "frac": by / avg_s / HBM_PEAK, "traffic": traffic.get(cat), "avg_us": avg_s * 1e6,
                           "total_ms": p["ms"], "launches": p["count"],
                           "per_launch": f"{by:.4e} algorithmic bytes"}
        return rl

    rl = rooflines(prof)
    rl_iso = rooflines(prof_iso)
    hbm = {c: v for c, v in rl.items() if v["bound"] == "hbm"}
    dom = max(hbm, key=lambda c: hbm[c]["total_ms"]) if hbm else None
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
                               f"{args.precision}, {args.streams} concurrent k-path segments",
                   "N": N, "nbands": m, "nk": nk, "tol": args.tol, "precision": args.precision,
                   "warm_start": args.warm, "guard": args.guard, "streams": args.streams,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        "roofline_source": "HIP events recorded around each launch on its own stream during the timed steps "
                           "(concurrent k-path segments overlap); kernels_isolated: the same from a "
                           f"single-stream pass over {min(args.roofline_nk, nk)} k-points after the timed steps",
        # the timed region's durations include the wait for CUs that the other
        # concurrent segments hold; the same kernel alone on the chip beside them
        "roofline": dict(rl[dom], kernel=dom,
                         single_stream={k: rl_iso[dom][k] for k in ("achieved", "frac", "avg_us")}
                         if dom in rl_iso else None) if dom else None,
        # the metric's second part: the fused stencil on a full block of the
        # workload's 16 bands in FP32 (one call: 204.5 MB at N = 64), alone on
        # the chip; beside it the FP64-arithmetic form the solver applies to
        # its FP32 W, and the solver's own soft-locked launches
        "stencil": stencil_object(stencil_direct(B, ctx, kpts[min(16, nk - 1)], m, N, torch),
                                  rl.get("stencil"), rl_iso.get("stencil")),
        "kernels": rl,
        "kernels_isolated": rl_iso,
        "iters_per_k": float(np.mean(iters)) if iters else None,
        "max_rel_resid": maxres,
        "converged_kpoints": ok,
        "total_kpoints": len(iters),
        "variants": variants,
        "tuning": B.mfd_tuning(ctx)[1],
    }
    if not args.no_cpu_baseline:
        kidx = min(16, len(kpts) - 1)
        line["cpu_baseline"] = cpu_baseline(eps, L, kpts[kidx], m, args.cpu_iters,
                                            float(np.mean(iters)) if iters else 1.0)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
