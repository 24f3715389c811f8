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
  roofline      - the dominant kernel (the largest share of the solve's
                  kernel time among the kernels that occupy the whole chip)
                  against its MI355X peak, from HIP events around each launch
                  in a single-stream pass over the first k-points after the
                  timed steps; roofline_check: the summed event time fits in
                  that pass's wall time;
  stencil       - the metric's second part: the fused stencil alone on full
                  16-band blocks rotated over a working set above the
                  Infinity Cache, FP32, FP32-storage/FP64-arithmetic and FP64;
                  precond the same for the FFT preconditioner;
  variants      - one timed step each of the plain FP64 solve, of a
                  32-crystal batch, of the learned warm start at N = 96 (with
                  the previous-k start and the untrained network beside it),
                  and of the band structures of Section 6's cells;
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
    ap.add_argument("--guard", type=int, default=4,
                    help="extra block columns beyond the bands (16 + 4 = 20 columns: fewest seconds per "
                         "k-point of guard 2..6 on the diamond N = 64 path)")
    ap.add_argument("--streams", type=int, default=12, help="k-path segments solved concurrently")
    ap.add_argument("--hard-lock", type=int, default=1, choices=[0, 1],
                    help="1: hard locking once at most 8 bands of a k-point iterate (opts.hard_lock)")
    ap.add_argument("--balance", type=int, default=0, choices=[0, 1],
                    help="1: a stream whose segment is done takes half of the busiest segment's remaining "
                         "k-points (opts.balance); 0: fixed segments")
    ap.add_argument("--cold-start", default="planewave", choices=["planewave", "random"],
                    help="start block of each segment's first k-point: the lowest transverse plane waves at k "
                         "(opts.cold_start = 1) or seeded random values")
    ap.add_argument("--warm", default="prev", choices=["prev", "learned"],
                    help="start block after a segment's first k-point: previous k, or the learned proposal")
    ap.add_argument("--tuning", default="",
                    help="JSON object of launch shapes to pin after the warm-up's autotuning (keys of "
                         "mfd_tuning, e.g. '{\"gram_workgroups\": 512}'); the others keep the tuned values")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the one-step comparison runs (FP64 solve, learned warm start)")
    ap.add_argument("--roofline-nk", type=int, default=6, help="k-points of the single-stream timing pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--learned-streams", type=int, default=4,
                    help="k-path segments of the learned-warm-start variant (N = 96, 100 k-points); long "
                         "segments give the network its training pairs")
    ap.add_argument("--profile-only", action="store_true", help="one short step, no JSON (for rocprofv3)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the single-stream pass the roofline object is taken from (for rocprofv3); "
                         "prints its JSON object")
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
T_START = time.perf_counter()


def progress(msg):
    """One line on stderr per finished piece of work (the JSON line goes to stdout)."""
    print(f"[bench {time.perf_counter() - T_START:7.1f} s] {msg}", file=sys.stderr, flush=True)
PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
KERNEL_SOURCES = {"update": ("gemm.hip", "lock.hip"), "gram": ("gemm.hip",), "stencil": ("stencil.hip",),
                  "precond": ("fft.hip",)}


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
        h = hashlib.sha256()   # over the category's source files, in order
        for name in src:
            with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2503_19379_amd", "csrc", name),
                      "rb") as f:
                h.update(f.read())
        digest = h.hexdigest()
        if fields.get("source_sha256") == digest and "traffic_bytes_per_launch" in fields:
            out[cat] = float(fields["traffic_bytes_per_launch"])
    return out


def batch_workers(args):
    return min(2 * args.streams, 16)


def batch_variant(B, args, torch, count):
    """Many crystals of uneven grids in one mfd_bands_batch call: 32 seeded
    random-field crystals (N = 24, 32, 48, 64 in turn), 8 k-points on
    Gamma-X-M-Gamma-R and 12 bands each, mixed precision, crystals handed to
    the workers in a queue.  Timed twice: with graph chunks (iterations
    replayed from captured HIP graphs, the host reading residuals between
    chunks) and host-stepped; each after an untimed call that sizes every
    crystal's workspace."""
    from paper_2503_19379_amd import workloads
    cfg = workloads.CONFIGS["random_batch"]
    crystals = workloads.random_batch_crystals(cfg["ncrys"], cfg["Ns"])
    ctxs = [B.mfd_build(N, 1.0, 2, eps) for N, eps in crystals]
    kp = workloads.kpath(cfg["path"], cfg["nk"])
    out = {"workload": f"{cfg['ncrys']} random-field crystals (correlation length 0.15, 30% eps 13 in 1), "
                       f"N in {cfg['Ns']}, {cfg['nk']} k-points on {cfg['path']}, {cfg['nbands']} bands, "
                       f"tol {cfg['tol']:g}, mixed precision"}
    for name, graph in (("graph", 1), ("host_stepped", 0)):
        o = B.default_opts(precision=1, warm_start=1, seed=0, guard=args.guard, max_iter=500, cold_start=cold(args),
                           streams=batch_workers(args), graph=graph)
        B.mfd_bands_batch(ctxs, [kp[:1]] * len(ctxs), cfg["nbands"], cfg["tol"], o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs, sts, status = B.mfd_bands_batch(ctxs, [kp] * len(ctxs), cfg["nbands"], cfg["tol"], o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok, iters, maxres = count([(None, st, status) for st in sts])
        syncs = sum(x["host_syncs"] for st in sts for x in st)
        out[name] = {"value": ok / dt, "unit": "k-points/s", "ms": dt * 1e3, "iters_per_k": float(np.mean(iters)),
                     "converged_kpoints": ok, "total_kpoints": len(iters), "max_rel_resid": maxres,
                     "host_syncs_per_iteration": syncs / max(1, sum(iters)), "workers": o.streams}
    for c in ctxs:
        c.close()
    out.update(value=out["graph"]["value"], unit="k-points/s")
    return out


def cold(args):
    return 1 if args.cold_start == "planewave" else 0


def gap_streams(args, N, mb):
    """Segments for a band-structure run: at most args.streams, and no more
    mixed-precision workspaces (V and U with 6 mb columns of n = 3 N^3 rows,
    in FP64 and again in FP32: 48 bytes per entry pair) than fit in 200 GB of
    HBM (6 at N = 150 with 12 columns)."""
    per = 3 * N ** 3 * 6 * mb * (2 * 16 + 2 * 8)
    return max(1, min(args.streams, int(200e9 // per)))


def band_gap_variant(B, args, torch):
    """Section 6.2's curved-interface cubic cell (sphere 0.345 + three
    cylinders 0.11, eps 13 in 1, M_0 set per edge) at the paper's N = 150: 10 bands along
    Gamma-X-M-Gamma-R-X-M-R with every symmetry point, the paper's tolerance
    1e-5, mixed precision, then the band-gap ratio.  One timed call after an
    untimed one at the first k-point."""
    from paper_2503_19379_amd import workloads
    cfg = workloads.CONFIGS["sc_sphere_cyl"]
    N = cfg["N"]
    kp = workloads.kpath_vertices(cfg["path"], cfg["nk"])
    ctx = B.mfd_build_mu(N, 1.0, 2, workloads.mu_sc_sphere_cylinders(N))
    o = B.default_opts(precision=1, warm_start=1, seed=0, guard=2, max_iter=500, cold_start=cold(args),
                       streams=gap_streams(args, N, cfg["nbands"] + 2))
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
            "gap_ratio_paper": cfg["gap_ratio_paper"], "N_paper": cfg["N_paper"], "segments": o.streams,
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
    structure on H'-Gamma-P-N-H at the paper's N = 150 and its gap ratio.
    (3) The lattice operator alone on a 12-band block at N = 120
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
                          "max_rel_resid": st[0]["max_rel_resid"], "status": status}
        if N == cfg["Ns"][-1]:
            out["lattice_operator"] = lattice_op_direct(B, ctx, kP[0], cfg["nbands"] + 2, N, torch)
        ctx.close()
    N = cfg["N_path"]
    ctx = B.mfd_build_lattice_mu(N, A, 2, workloads.mu_bcc_gyroid(N))
    kp = workloads.kpath_vertices(cfg["path"], cfg["nk"], points=workloads.bcc_points())
    o = B.default_opts(precision=1, warm_start=1, seed=0, guard=2, max_iter=500, cold_start=cold(args),
                       streams=gap_streams(args, N, cfg["nbands"] + 2))
    B.mfd_bands(ctx, kp[:1], cfg["nbands"], cfg["tol"], o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, st, status = B.mfd_bands(ctx, kp, cfg["nbands"], cfg["tol"], o)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ratio, below = B.mfd_gap_ratio(ev, kp)
    ok = sum(1 for x in st if x["max_rel_resid"] <= cfg["tol"])
    out[f"path_N{N}"] = {"value": ok / dt, "unit": "k-points/s", "ms": dt * 1e3, "kpoints": len(kp),
                         "converged_kpoints": ok, "gap_ratio": ratio, "gap_above_band": below,
                         "gap_ratio_paper": cfg["gap_ratio_paper"], "N_paper": cfg["N_paper"],
                         "segments": o.streams}
    ctx.close()
    return out


def _rotating_blocks(torch, m, N, dtype, count):
    g = torch.Generator(device="cuda").manual_seed(0)
    return [torch.randn((m, 3, N, N, N), dtype=dtype, device="cuda", generator=g) for _ in range(count)]


def _timed_calls(torch, s, calls, reps):
    """Mean duration of `reps` passes over `calls` (back-to-back launches on
    stream s) between HIP events recorded on s, after one untimed pass."""
    for c in calls:
        c()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        for c in calls:
            c()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / (reps * len(calls))


def stencil_direct(B, ctx, k, m, N, torch, min_ws=512e6, reps=10):
    """The fused stencil alone on full blocks of m bands (no soft locking),
    nothing else on the chip.  The calls rotate over enough distinct (X, Y)
    block pairs that the working set is at least min_ws bytes (above the
    256 MB Infinity Cache), so every call streams from HBM.  Algorithmic
    bytes per call: X read and Y written once (2 x 24 N^3 m bytes in FP32
    storage, 2 x 48 in FP64) plus M_0 once (FP32 copy 12 N^3, FP64 24 N^3);
    the neighbour values come from registers, LDS or cache.  Three forms:
    FP32 storage and arithmetic; FP32 storage with FP64 arithmetic (what the
    mixed-precision solve applies to its search directions); FP64 (the FP64
    solve)."""
    n3 = N ** 3
    s = torch.cuda.Stream()
    out = {}
    for name, dtype, f64, by in (("fp32", torch.complex64, False, 48.0 * n3 * m + 12.0 * n3),
                                 ("fp32_storage_fp64_arith", torch.complex64, True, 48.0 * n3 * m + 24.0 * n3),
                                 ("fp64", torch.complex128, False, 96.0 * n3 * m + 24.0 * n3)):
        per_pair = 2 * m * 3 * n3 * (8 if dtype == torch.complex64 else 16)
        npair = max(2, int(np.ceil(min_ws / per_pair)))
        X = _rotating_blocks(torch, m, N, dtype, npair)
        Y = [torch.empty_like(x) for x in X]
        calls = [(lambda x=x, y=y: B.mfd_op_apply(ctx, k, x, y, stream=s.cuda_stream, fp64_arith=f64))
                 for x, y in zip(X, Y)]
        avg_s = _timed_calls(torch, s, calls, reps)
        out[name] = {"achieved": by / avg_s / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": by / avg_s / HBM_PEAK, "avg_us": avg_s * 1e6, "bytes_per_call": by,
                     "working_set_bytes": npair * per_pair + (24 if f64 or dtype == torch.complex128 else 12) * n3,
                     "blocks_rotated": npair, "nbands": m, "N": N, "calls": reps * npair}
        del X, Y, calls
        torch.cuda.synchronize()
    return out


def precond_direct(B, ctx, k, m, N, torch, min_ws=512e6, reps=10):
    """The FFT preconditioner alone on full FP32 blocks of m bands, in place,
    rotating over enough distinct blocks for a working set of at least
    min_ws bytes.  Algorithmic bytes: one read and one write of the block
    (48 B per cell and band), the single-pass minimum; the design makes three
    passes (x-y plane FFT, z FFT with the 3 x 3 solve, inverse plane FFT), so
    the bytes it moves are three times that."""
    n3 = N ** 3
    s = torch.cuda.Stream()
    per = m * 3 * n3 * 8
    nblk = max(2, int(np.ceil(min_ws / per)))
    X = _rotating_blocks(torch, m, N, torch.complex64, nblk)
    calls = [(lambda x=x: B.mfd_precond_solve(ctx, k, x, x, stream=s.cuda_stream)) for x in X]
    avg_s = _timed_calls(torch, s, calls, reps)
    by = 48.0 * n3 * m
    del X, calls
    torch.cuda.synchronize()
    return {"achieved": by / avg_s / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": by / avg_s / HBM_PEAK,
            "moved_three_pass_GBps": 3 * by / avg_s / 1e9, "moved_three_pass_frac": 3 * by / avg_s / HBM_PEAK,
            "avg_us": avg_s * 1e6, "bytes_per_call": by, "working_set_bytes": nblk * per, "blocks_rotated": nblk,
            "nbands": m, "N": N, "calls": reps * nblk, "form": "FP32, in place"}


def learned_variant(B, args, torch):
    """The learned-warm-start workload: diamond cell at N = 96 (2,654,208
    unknowns), 100 k-points on Gamma-X-M-Gamma-R-X, 20 bands, mixed
    precision, tol 1e-8.  Each k-path segment is solved with the previous-k
    start, with the learned proposal (network trained along the path), and
    with the untrained network (learn_steps = 0: the aligned-subspace
    extrapolation it starts from).  One timed call each after an untimed one
    that sizes the workspaces."""
    from paper_2503_19379_amd import workloads
    cfg = workloads.CONFIGS["diamond_n96"]
    N, m = cfg["N"], cfg["nbands"]
    kp = workloads.kpath(cfg["path"], cfg["nk"])
    ctx = B.mfd_build(N, 1.0, 2, workloads.crystal_eps(cfg["eps"], N))
    guard = max(0, min(args.guard, B.max_block() - m))
    out = {"workload": f"diamond cell, N = {N} ({3 * N ** 3} unknowns), {len(kp)} k-points on {cfg['path']}, "
                       f"{m} bands, tol {cfg['tol']:g}, mixed precision, guard {guard}, "
                       f"{args.learned_streams} k-path segments"}
    for name, warm, steps in (("previous_k", 1, 30), ("learned", 2, 30), ("untrained", 2, 0)):
        o = B.default_opts(precision=1, warm_start=warm, learn_steps=steps, seed=0, guard=guard, max_iter=500,
                           cold_start=cold(args),
                           streams=args.learned_streams)
        B.mfd_bands(ctx, kp[:args.learned_streams], m, cfg["tol"], o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, st, status = B.mfd_bands(ctx, kp, m, cfg["tol"], o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = sum(1 for x in st if x["max_rel_resid"] <= cfg["tol"] and x["spurious"] == 0)
        out[name] = {"value": ok / dt, "unit": "k-points/s", "ms": dt * 1e3,
                     "iters_per_k": float(np.mean([x["iters"] for x in st])),
                     "iters_total": int(sum(x["iters"] for x in st)), "converged_kpoints": ok,
                     "total_kpoints": len(st),
                     "proposals_used": int(sum(1 for x in st if warm == 2 and not x["used_fallback"]))}
    ctx.close()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(eps, L, kpts, kidx, m, guard, gpu_iters_per_k):
    """The FP64 oracle as it stands, on this host: at each k-index of kidx
    (cold start, seed 0, the same block of m + guard columns), its LOBPCG is
    timed for 1 and for 2 iterations; the difference is one iteration, the
    rest the start-up (FFT symbol inverses, QR, first operator application).
    Seconds per k-point = start-up + one iteration x the GPU run's mean
    iterations per k-point.  FFTs run on os.cpu_count() threads, BLAS on its
    own pool; both are recorded."""
    from oracle import lobpcg as olob
    from oracle import mfd as omfd
    from paper_2503_19379_amd import workloads
    ncpu = os.cpu_count() or 1
    omfd.FFT_WORKERS = ncpu
    N = eps.shape[0]
    n = 3 * N ** 3
    h = L / N
    mu = omfd.mu_from_eps(eps)
    X0 = workloads.start_block(m + guard, N, 0).reshape(m + guard, n).T
    per_iter, startup = [], []
    t_all = time.perf_counter()
    for ki in kidx:
        k = kpts[ki]
        g = omfd.gamma_rule(N, L, k)
        c = omfd.shift_rule(L, k)
        times = []
        for iters in (1, 2):
            t0 = time.perf_counter()
            Pinv = np.linalg.inv(omfd.precond_matrices(N, L, k, g, 2, c))
            A = lambda X: omfd.apply_op(X.T.reshape(-1, 3, N, N, N), mu, k, h, g, 2, c).reshape(-1, n).T
            T = lambda R: omfd.precond_solve(R.T.reshape(-1, 3, N, N, N), N, L, k, g, 2, c,
                                             Pinv=Pinv).reshape(-1, n).T
            olob.lobpcg(A, T, X0, 1e-8, maxiter=iters)
            times.append(time.perf_counter() - t0)
        per_iter.append(max(times[1] - times[0], 0.0))
        startup.append(times[0] - per_iter[-1])
        progress(f"CPU oracle at k-index {ki}: {times[0]:.1f} s (1 iteration), {times[1]:.1f} s (2)")
    wall = time.perf_counter() - t_all
    s_per_k = float(np.mean(startup) + np.mean(per_iter) * gpu_iters_per_k)
    try:
        from threadpoolctl import threadpool_info
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except ImportError:
        blas = None
    return {"value": 1.0 / s_per_k, "unit": "k-points/s", "cores": ncpu, "kind": "oracle",
            "s_per_kpoint": s_per_k, "s_per_iteration": float(np.mean(per_iter)),
            "startup_s": float(np.mean(startup)), "nproc": ncpu, "cpu_model": cpu_model(),
            "fft_workers": ncpu, "blas_threads": blas,
            "sample": f"oracle LOBPCG at k-indices {list(kidx)} of the same path (cold start, seed 0, "
                      f"{m} + {guard} columns), 1 and 2 iterations each ({wall:.1f} s in all); seconds per "
                      f"k-point = start-up + one iteration x {gpu_iters_per_k:.1f} (the GPU run's mean "
                      f"iterations per k-point)"}


def kernel_table(prof, wall_s=None):
    """Per-kernel average durations and rates from the library's HIP-event
    timing.  Gram: flops (8 n K (K+1) per launch) against the FP64 MFMA peak
    (its arithmetic as built); the others: algorithmic bytes against HBM."""
    rl = {}
    for cat in ("stencil", "precond", "gram", "update", "rr", "other"):
        p = prof[cat]
        if p["count"] == 0 or p["ms"] == 0:
            continue
        avg_s = p["ms"] / p["count"] * 1e-3
        per = p["bytes"] / p["count"]
        e = {"avg_us": avg_s * 1e6, "total_ms": p["ms"], "launches": p["count"]}
        if cat == "rr":
            e.update(bound="latency", note="one workgroup (one CU); overlaps other segments' kernels")
        elif cat == "other":
            e.update(bound="latency", note="fixed-order sums of the Gram tiles and of the update's column norms; "
                     "under hard locking the projections of W (and P) against the locked vectors")
        elif cat == "gram":
            e.update(bound="mfma", achieved=per / avg_s / 1e12, peak=FP64_PEAK / 1e12, unit="TFLOP/s",
                     frac=per / avg_s / FP64_PEAK, per_launch=per,
                     per_launch_note="8 n K (K+1) flops for the launch's basis of K = mb + 2 na columns "
                                     "(S^H S and S^H AS, Hermitian halves); mean over launches")
        else:
            e.update(bound="hbm", achieved=per / avg_s / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s",
                     frac=per / avg_s / HBM_PEAK, per_launch=per, per_launch_note="algorithmic bytes")
        rl[cat] = e
    total = sum(v["total_ms"] for v in rl.values())
    for v in rl.values():
        v["share"] = v["total_ms"] / total if total else None
    return rl, total


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

    def make_opts(precision, warm, streams=args.streams):
        return B.default_opts(precision=1 if precision == "mixed" else 0, warm_start=2 if warm == "learned" else 1,
                              seed=0, guard=args.guard, max_iter=500, streams=streams, cold_start=cold(args),
                              balance=args.balance if warm != "learned" else 0, hard_lock=args.hard_lock)

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

    nk_iso = max(1, min(args.roofline_nk, nk))

    def single_stream_pass():
        """The kernels without the overlap of concurrent segments: one stream
        over the first k-points of the path, HIP events around every launch on
        that stream.  Returns (per-kernel table, wall seconds, summed event time)."""
        B.mfd_profile(ctx, True)
        o1 = make_opts(args.precision, "prev", streams=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.mfd_bands(ctx, kpts[:nk_iso], m, args.tol, o1)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = B.mfd_profile_read(ctx)
        B.mfd_profile(ctx, False)
        table, total_ms = kernel_table(prof)
        return table, wall, total_ms

    if args.lattice_only:
        print(json.dumps(lattice_only(B, torch)))
        if args.copy_calib:
            copy_calibration()
        return
    if args.stencil_only:
        print(json.dumps({"stencil": stencil_direct(B, ctx, kpts[min(16, nk - 1)], m, N, torch),
                          "precond": precond_direct(B, ctx, kpts[min(16, nk - 1)], m, N, torch)}))
        if args.copy_calib:
            copy_calibration()
        return
    if args.profile_only:
        step()
        torch.cuda.synchronize()
        if args.copy_calib:
            copy_calibration()
        return
    if args.roofline_only:
        B.mfd_bands(ctx, kpts[:nk_iso], m, args.tol, make_opts(args.precision, "prev", streams=1))
        table, wall, total_ms = single_stream_pass()
        print(json.dumps({"kernels_isolated": table, "wall_ms": wall * 1e3, "event_ms": total_ms}))
        if args.copy_calib:
            copy_calibration()
        return
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        progress(f"warm-up step {i + 1} of {args.warmup} done")
    if args.tuning:
        if not B.mfd_tuning(ctx)[0]:
            step()   # no warm-up step: let the autotuner run once
        shapes = B.mfd_tuning(ctx)[1]
        shapes.update(json.loads(args.tuning))
        B.mfd_set_tuning(ctx, shapes)
    # Per-kernel durations during the timed steps: HIP events recorded by the
    # library around each launch on the stream it is launched on.
    B.mfd_profile(ctx, True)
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(step())
        progress(f"timed step {i + 1} of {args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = B.mfd_profile_read(ctx)
    B.mfd_profile(ctx, False)
    iso, iso_wall, iso_event_ms = single_stream_pass()
    progress("single-stream pass done")

    if args.verbose:
        for ev, st, status in results:
            for i, s in enumerate(st):
                print(f"k{i:3d} {np.array2string(kpts[i], precision=3)} iters={s['iters']:4d} "
                      f"res={s['max_rel_resid']:.2e} dbl={s['gamma_doublings']} spur={s['spurious']} "
                      f"ms={s['ms']:.1f} ev0={ev[i][0]:.6f} ev15={ev[i][-1]:.6f}", file=sys.stderr)
    ok, iters, maxres = count(results)
    value = ok / dt
    # iterations at the segments' first k-points (cold starts) and at the
    # warm-started rest, and the k-points that left the mixed iteration or
    # rejected a step
    cold_it = [s["iters"] for _, st, _ in results for s in st if s["segment_start"]]
    warm_it = [s["iters"] for _, st, _ in results for s in st if not s["segment_start"]]
    allst = [s for _, st, _ in results for s in st]
    kstats = {"segment_starts": len(cold_it),
              "iters_cold_start_mean": float(np.mean(cold_it)) if cold_it else None,
              "iters_warm_start_mean": float(np.mean(warm_it)) if warm_it else None,
              "fp64_fallback_kpoints": int(sum(s["fp64_fallback"] for s in allst)),
              "rejected_steps": int(sum(s["rejected_steps"] for s in allst)),
              "gamma_doublings": int(sum(s["gamma_doublings"] for s in allst)),
              "discarded_bands": int(sum(s["discarded"] for s in allst))}

    # One-step comparison runs on the same GPU (each after an untimed call
    # that sizes its workspaces).
    variants = {}
    if not args.no_variants:
        for name, prec, warm in (("fp64_prev", "fp64", "prev"),):
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
            progress(f"variant {name} done")
        for name, fn in (("random_batch", lambda: batch_variant(B, args, torch, count)),
                         ("learned_n96", lambda: learned_variant(B, args, torch)),
                         ("sc_sphere_cyl_gap", lambda: band_gap_variant(B, args, torch)),
                         ("bcc_gyroid", lambda: gyroid_variant(B, args, torch))):
            variants[name] = fn()
            progress(f"variant {name} done")
    n = 3 * N ** 3
    traffic = measured_traffic(args.workload, args.precision)
    for cat, v in iso.items():
        if v.get("bound") in ("hbm", "mfma"):
            v["traffic"] = traffic.get(cat)
    timed, timed_total = kernel_table(prof)
    # the dominant kernel: the largest share of the single-stream time among
    # the kernels that occupy the whole chip (the Rayleigh-Ritz step runs on
    # one CU and the sums are latency-bound)
    chip = {c: v for c, v in iso.items() if v.get("bound") in ("hbm", "mfma")}
    dom = max(chip, key=lambda c: chip[c]["total_ms"]) if chip else None
    fits = iso_event_ms <= iso_wall * 1e3 * 1.001
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
                   "warm_start": args.warm, "cold_start": args.cold_start, "guard": args.guard, "streams": args.streams,
                   "balance": args.balance, "hard_lock": args.hard_lock,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        # the kernels alone: a single-stream pass over the first k-points of
        # the path after the timed steps, HIP events on the launching stream
        "roofline": dict(chip[dom], kernel=dom, source=f"single-stream pass over {nk_iso} k-points after the "
                         "timed steps; HIP events around each launch on its stream") if dom else None,
        "roofline_check": {"event_ms": iso_event_ms, "wall_ms": iso_wall * 1e3, "events_fit_in_wall": fits},
        # the metric's second part: the fused stencil (and the FFT
        # preconditioner) alone on full blocks, working sets above the
        # Infinity Cache
        "kernels_isolated": iso,
        # in the timed steps the concurrent segments overlap: a launch's event
        # time includes the wait for CUs held by other segments, so these are
        # shares of stream time, not kernel rates
        "kernels_timed_region_share": {c: {"share": v["share"], "launches": v["launches"]}
                                       for c, v in timed.items()},
        "iters_per_k": float(np.mean(iters)) if iters else None,
        "kpoint_stats": kstats,
        "max_rel_resid": maxres,
        "converged_kpoints": ok,
        "total_kpoints": len(iters),
        "variants": variants,
        "tuning": B.mfd_tuning(ctx)[1],
    }
    line["stencil"] = stencil_direct(B, ctx, kpts[min(16, nk - 1)], m, N, torch)
    line["precond"] = precond_direct(B, ctx, kpts[min(16, nk - 1)], m, N, torch)
    progress("stencil and preconditioner on full blocks done")
    if not args.no_variants:
        s96 = workloads.CONFIGS["diamond_n96"]
        ctx96 = B.mfd_build(s96["N"], 1.0, 2, workloads.crystal_eps(s96["eps"], s96["N"]))
        k96 = workloads.kpath(s96["path"], s96["nk"])[16]
        line["stencil_n96_20bands"] = stencil_direct(B, ctx96, k96, s96["nbands"], s96["N"], torch)
        ctx96.close()
        progress("stencil on the N = 96, 20-band block done")
    if not args.no_cpu_baseline:
        kidx = [i for i in (0, 16, 32, 48) if i < len(kpts)]
        line["cpu_baseline"] = cpu_baseline(eps, L, kpts, kidx, m, args.guard,
                                            float(np.mean(iters)) if iters else 1.0)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
