#!/usr/bin/env python3
"""Throughput of the narrow-band Bayesian SDF solve on one MI355X.

One step is one pass of the whole hot path over the 512^3 union scene (3
spheres, a rounded box and a torus; 2 mm voxels, +-4 voxel band, 120 views at
640x480 on a 1.2 m hemisphere, sigma(z) depth noise), the full-pass
configuration:
  coarse TSDF + band + key -> index map + neighbours  ->  assembly of Lambda,
  b, diag(Q)  ->  features + network (learned start)  ->  mixed-precision
  Jacobi-PCG for the mean from the learned start (tol 1e-6)  ->  32-probe
  Hutchinson variance as one mixed-precision block-PCG from the learned
  log-variance (tol 1e-6)  ->  NBV scoring of 512 candidate poses (160x120
  rays each) with argmax.
Inputs are synthetic and resident in device memory before timing starts.

Printed: one JSON line with the metric (band voxel-PCG-iterations per second
of step time), the roofline of the solver iteration in its algorithmic bytes
per voxel-column-iteration (block A + B + verify over their event-timed
average durations), per-kernel rooflines, the 256^3 FP64 step, the
learned/batched/mixed vs plain FP64 time-to-tolerance comparison, the solver
kernels on a band far larger than the Infinity Cache, and the FP64 CPU oracle
timed on a bounded sample of the same workload at one thread and at every
host core.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP64 vector issue rate without FMA: 256 CUs x 64 lanes x 2.4 GHz.
FP64_ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# HBM traffic of the roofline kernel, from two rocprofv3 --pmc runs of this
# bench (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) scaled by what the same
# counters read for a plain copy of known size (bench.py --copy-calibration).
# The figures hold only for the kernel sources they were taken from (hashes).
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
COPY_BYTES = 1 << 30


def copy_calibration():
    """A plain streaming kernel over COPY_BYTES: b = a * 1 reads and writes that
    many bytes (torch's elementwise kernel)."""
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "launches": 3}), flush=True)


def measured_traffic(kernel, workload):
    """HBM bytes per launch of the kernel timed as `kernel` on `workload` from
    the committed counters, or None if there are none or its source changed
    since."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        rec = json.load(f)
    entry = rec.get("kernels", {}).get(kernel)
    if entry is None or entry.get("workload") != workload:
        return None
    for src, digest in entry["sources"].items():
        with open(os.path.join(ROOT, src), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    fetch = entry["fetch_kib_per_dispatch"] * 1024 * rec["copy"]["fetch_factor"]
    write = entry["write_kib_per_dispatch"] * 1024 * rec["copy"]["write_factor"]
    return fetch + write


# Operations per fused voxel-view of the coarse TSDF (FP64 projection, two
# divisions, truncation, running sum) and per screening test of a (box, view)
# pair, the box being a super tile, a block tile or a 4^3 cell: one FP64 corner transform
# (27), box edges and Z range (22), 36 FP64 corner adds, 8 FP32 projections of
# 12 operations (96), pixel range and pyramid bounds (31), final tests (5),
# counted arithmetic, min/max, compare and convert operations alike.
TSDF_OPS_PER_VOXEL_VIEW = 35
TSDF_OPS_PER_CELL_VIEW = 217


def algorithmic_work(name, N, K, T, G, P, fp64=True, voxel_views=None, box_tests=None, warm=False,
                     estimate=False, tile_tests=None, assembly_views=None):
    """(amount, unit, bound) of one launch of a timed kernel.  warm: the probe
    solve starts from the log-variance start +-w (w per row) rather than 0.
    estimate: the verify pass also formed the variance estimate s (8 B per row
    out; the separate estimate pass then had nothing to do)."""
    s = 8 if fp64 else 4
    if name == "pcg_A":      # nbr, diag, z, p_old -> p_new, q
        return N * (24 + 5 * s), "B", "hbm"
    if name == "pcg_B":      # dinv, p, q, x, r -> x, r, z
        return N * 8 * s, "B", "hbm"
    if name == "block_A":    # nbr, diag; per column zz, p_old -> p_new, q
        return N * (24 + s + 4 * K * s), "B", "hbm"
    if name == "block_B":    # dinv; per column p, q, x, r -> x, r, zz
        return N * (s + 7 * K * s), "B", "hbm"
    if name == "block_A_first":  # first iteration: zz in, q out (p_0 = zz is used in place: no p_old, no p_new)
        return N * (24 + s + 2 * K * s), "B", "hbm"
    if name == "block_B_first":  # first iteration: x not read (it is 0, or the float correction's 0);
        # r not read either in FP64 from zero (regenerated from the probe signs)
        return N * (s + (6 if (warm or not fp64) else 5) * K * s), "B", "hbm"
    if name == "block_verify":   # FP64 residual norms: nbr, diag, the probe signs (K/8 B); per column
        # x64 in FP64; under mixed precision the float correction, over an FP64 part that is the
        # start (w per row, or zero) until a column's first restart
        est = 8 if estimate else 0
        if fp64:
            return N * (24 + 8 + K / 8 + 8 * K + est), "B", "hbm"
        return N * (24 + 8 + K / 8 + (8 if warm else 0) + 4 * K + est), "B", "hbm"
    if name == "block_start_res":  # from +-w: nbr, diag, w, signs in; per column r, zz out (+ x64 in FP64)
        return N * (24 + 8 + 8 + K / 8 + 2 * K * s + (8 * K if fp64 else 0)), "B", "hbm"
    # block_residual and pcg_residual time full passes (a start residual) and
    # checks that find nothing to do under one label: no per-launch roofline
    # screening: one super tile test per (32x16x16 super tile, view of the first
    # 256), block tile tests for the super tiles' undecided views, then cell
    # tests (all counted by the kernels but the first)
    super_tests = (-(-G // 32)) * (-(-G // 16)) ** 2 * min(T, 256)
    if name == "tsdf_count":  # fused voxel-views (counted by the kernel)
        vv = G ** 3 * T if voxel_views is None else voxel_views
        return vv * TSDF_OPS_PER_VOXEL_VIEW, "flop", "alu"
    if name == "super_screen":
        return super_tests * TSDF_OPS_PER_CELL_VIEW, "flop", "alu"
    if name == "tile_screen" and tile_tests is not None:
        return (tile_tests - super_tests) * TSDF_OPS_PER_CELL_VIEW, "flop", "alu"
    if name == "cell_screen" and box_tests is not None and tile_tests is not None:
        return (box_tests - tile_tests) * TSDF_OPS_PER_CELL_VIEW, "flop", "alu"
    if name == "assemble":  # the (voxel, view) pairs it goes through (its view masks skip the rest)
        return (N * T if assembly_views is None else assembly_views) * 45, "flop", "alu"
    return None


def iteration_bytes(K, fp64):
    """Algorithmic bytes of one CG iteration per unit of work: a band voxel for
    one right-hand side (FP64 2-pass 120 B, mixed 72 B), or a voxel-column of a
    K-column block solve (10 s + 32 / K with s the vector element size: the
    matrix, 24 B of neighbours and the diagonal, amortised over the columns)."""
    s = 8 if fp64 else 4
    if K == 1:
        return 120 if fp64 else 72
    return 10 * s + 32.0 / K


SOLVER_ITERATION = ("block_A", "block_A_first", "block_B", "block_B_first", "block_verify")


def solver_roofline(kernels, N, K, fp64, col_iters):
    """The block solve's iteration against HBM: voxel-column-iterations x the
    per-unit algorithmic bytes over the summed busy time of the kernels one
    iteration runs (A, B and the FP64 verify pass, first-iteration variants
    included), all from HIP events on the library stream."""
    busy_ms = sum(kernels[k]["total_ms"] for k in SOLVER_ITERATION if k in kernels)
    if busy_ms <= 0 or col_iters <= 0:
        return None
    per_unit = iteration_bytes(K, fp64)
    amount = N * col_iters * per_unit
    ach = amount / (busy_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "kernel": "+".join(k for k in SOLVER_ITERATION if k in kernels),
            "unit_of_work": "voxel-column-iteration", "bytes_per_unit": per_unit,
            "units": N * col_iters, "busy_ms": busy_ms}


def run_gpu(args):
    import torch
    import paper_2602_19697_amd as bf
    from synth import make_workload

    dev = torch.device("cuda:0")
    t0 = time.time()
    wl = make_workload(args.workload, device=dev)
    log(f"[bench] workload {wl.name}: G={wl.G} views={wl.T} {wl.cam.width}x{wl.cam.height} "
        f"rendered in {time.time() - t0:.1f}s")
    depth = torch.from_numpy(wl.depth).to(dev)
    poses = torch.from_numpy(np.ascontiguousarray(wl.poses)).to(dev)
    cands_np = wl.candidates()
    cands = torch.from_numpy(np.ascontiguousarray(cands_np)).to(dev)
    grid = bf.grid_struct(wl.G, wl.h, wl.origin, wl.tau, wl.band)
    noise = bf.noise_struct(*wl.noise)
    # bands and systems from torch's caching allocator (the binding's default) or the library's pool
    ctx = bf.Context(dev, allocator="torch" if args.allocator == "torch" else None)
    K = args.probes

    prec = bf.L.BF_PREC_FP64 if args.precision == "fp64" else bf.L.BF_PREC_MIXED
    params = None
    if args.learned:
        path = _weights(wl.lam)
        if path is None:
            raise SystemExit(f"--learned: no trained warm start for lambda={wl.lam}")
        params = torch.from_numpy(np.load(path)).to(dev)

    def step():
        band = ctx.bf_build_band(grid, wl.cam, depth, poses)
        sys_ = ctx.bf_assemble(band, wl.cam, depth, poses, noise, wl.lam, wl.eps)
        if params is not None:  # learned start: features -> network -> x0 and log-variance
            x0, lv = ctx.bf_warm_start(sys_, params)  # features computed in the network's pass
        else:
            x0 = lv = None
        mu, rep = ctx.bf_pcg_solve(sys_, args.tol, precision=prec, x0=x0)
        s, prep = ctx.bf_diag_estimate(sys_, K, 0, args.tol, precision=prec, logvar=lv)
        scores, best = ctx.bf_nbv_score(band, mu, s, cands, wl.ray_cam)
        out = dict(N=band.n, iters=rep["iters"], probe_iters=prep["iters"], walk_steps=ctx.bf_nbv_walk_steps(),
                   tsdf_voxel_views=band.info()["tsdf_voxel_views"], tsdf_box_tests=band.info()["tsdf_box_tests"],
                   tsdf_tile_tests=band.info()["tsdf_tile_tests"],
                   work=band.n * (rep["col_iters"] + prep["col_iters"]), best=best,
                   probe_col_iters=prep["col_iters"], mean_col_iters=rep["col_iters"],
                   rel_res=rep["rel_res"], probe_rel_res=prep["rel_res"])
        sys_.free()
        band.free()
        return out

    for _ in range(args.warmup):
        info = step()
    torch.cuda.synchronize()
    # per-kernel HIP events cost host time at every launch, so they run on the
    # last timing_steps steps of the timed region only
    timing_steps = max(1, min(args.timing_steps, args.steps))
    t_start = time.perf_counter()
    works = []
    for i in range(args.steps):
        if i == args.steps - timing_steps:
            ctx.bf_set_timing(True)
        info = step()
        works.append(info["work"])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ctx.bf_set_timing(False)
    timings = ctx.bf_get_timings()
    log(f"[bench] {args.steps} steps in {t_total:.3f}s; N={info['N']} iters={info['iters']} "
        f"probe iters={info['probe_iters']} best={info['best']}")
    ms_step = 1e3 * t_total / args.steps
    value = sum(works) / t_total
    # the (voxel, view) pairs the assembly goes through, from one more build
    # and assembly after the timed region (the count needs a host read-back)
    b_x = ctx.bf_build_band(grid, wl.cam, depth, poses)
    s_x = ctx.bf_assemble(b_x, wl.cam, depth, poses, noise, wl.lam, wl.eps)
    info["assembly_views"] = s_x.assembly_views()
    s_x.free()
    b_x.free()

    # kernel table and the dominant kernel's roofline
    kernels = {}
    for name, (launches, ms) in sorted(timings.items(), key=lambda kv: -kv[1][1]):
        kernels[name] = {"launches": launches, "avg_us": 1e3 * ms / max(launches, 1), "total_ms": ms,
                         "share_of_step": ms / timing_steps / ms_step}
    P = 1
    while P < wl.G:
        P *= 2
    rooflines = {}
    # the verify pass formed the estimate when the estimate pass never ran (or found it done)
    estimate = "block_verify" in kernels and "hutch_final" not in kernels
    for name, kt in kernels.items():
        w = algorithmic_work(name, info["N"], K, wl.T, wl.G, P, fp64=(args.precision == "fp64"),
                             voxel_views=info["tsdf_voxel_views"], box_tests=info["tsdf_box_tests"],
                             tile_tests=info["tsdf_tile_tests"], assembly_views=info["assembly_views"],
                             warm=args.learned, estimate=estimate)
        if w is None:
            continue
        amount, unit, bound = w
        avg_s = kt["avg_us"] * 1e-6
        if unit == "B":
            ach = amount / avg_s / 1e9
            rooflines[name] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": ach / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": amount,
                               "traffic": measured_traffic(name, wl.name)}
        else:
            ach = amount / avg_s / 1e12
            rooflines[name] = {"bound": "alu", "achieved": ach, "peak": FP64_ALU_PEAK_TOPS,
                               "unit": "TFLOP/s", "frac": ach / FP64_ALU_PEAK_TOPS,
                               "algorithmic_flops_per_launch": amount, "traffic": measured_traffic(name, wl.name)}
    dominant = next(iter(kernels)) if kernels else None
    # the block solve's iteration in the section 8(d) unit, over the timed steps' launches
    solver = solver_roofline(kernels, info["N"], K, args.precision == "fp64", info["probe_col_iters"] * timing_steps)
    return dict(ctx=ctx, wl=wl, depth=depth, poses=poses, cands=cands, grid=grid, noise=noise,
                info=info, value=value, ms_step=ms_step, kernels=kernels, rooflines=rooflines,
                dominant=dominant, solver_roofline=solver, precision=args.precision, learned=args.learned,
                K=K, tol=args.tol, steps=args.steps, timing_steps=timing_steps)


def _weights(lam):
    from paper_2602_19697_amd import learned
    try:
        path = learned.weights_path(lam)
    except KeyError:
        return None
    return path if os.path.exists(path) else None


def _timed(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = fn()
    torch.cuda.synchronize()
    return r, 1e3 * (time.perf_counter() - t0) / reps


def time_to_tol(g, args, lam=None):
    """Mean plus K-probe variance to relative residual 1e-6 on the bench scene
    with prior strength lam (see compare_solvers)."""
    ctx, wl = g["ctx"], g["wl"]
    lam = wl.lam if lam is None else lam
    band = ctx.bf_build_band(g["grid"], wl.cam, g["depth"], g["poses"])
    sys_ = ctx.bf_assemble(band, wl.cam, g["depth"], g["poses"], g["noise"], lam, wl.eps)
    out = compare_solvers(ctx, sys_, lam, args.probes)
    sys_.free()
    band.free()
    return out


def compare_solvers(ctx, sys_, lam, K, reps=3, plain_reps=None):
    """Time to 1e-6 for the mean and the K-probe variance of one system: plain
    FP64 (mean PCG + K sequential one-probe solves, all from zero) against the
    block FP64 solve, the block mixed solve, and, where a network was trained
    for lam, the learned start (features + network, then mixed PCG from x0 and
    the mixed block solve from the predicted log-variance)."""
    import torch
    import paper_2602_19697_amd as bf
    tol = 1e-6
    FP64, MIXED = bf.L.BF_PREC_FP64, bf.L.BF_PREC_MIXED

    def plain():
        _, r = ctx.bf_pcg_solve(sys_, tol, precision=FP64)
        its = [r["iters"], 0]
        for k in range(K):
            _, pr = ctx.bf_diag_estimate(sys_, 1, 1000 + k, tol, precision=FP64)
            its[1] += pr["iters"]
        return its

    def block(prec):
        def run():
            _, r = ctx.bf_pcg_solve(sys_, tol, precision=prec)
            _, pr = ctx.bf_diag_estimate(sys_, K, 0, tol, precision=prec)
            return [r["iters"], pr["col_iters"]]
        return run

    variants = [("plain_fp64", plain), ("batched_fp64", block(FP64)), ("batched_mixed", block(MIXED))]
    params = None
    path = _weights(lam)
    if path is not None:
        params = torch.from_numpy(np.load(path)).to(ctx.device)

        def learned():
            x0, lv = ctx.bf_warm_start(sys_, params)  # features computed in the network's pass
            _, r = ctx.bf_pcg_solve(sys_, tol, precision=MIXED, x0=x0)
            _, pr = ctx.bf_diag_estimate(sys_, K, 0, tol, precision=MIXED, logvar=lv)
            return [r["iters"], pr["col_iters"]]
        variants.append(("learned_batched_mixed", learned))
    out = {"lambda": lam, "tol": tol, "probes": K}
    for name, fn in variants:
        its, ms = _timed(fn, plain_reps if (plain_reps and name == "plain_fp64") else reps)
        out[name + "_ms"] = ms
        out[name + "_iters"] = {"mean": its[0], "probe_columns": its[1]}
    out["speedup_batching"] = out["plain_fp64_ms"] / out["batched_fp64_ms"]
    out["speedup_precision"] = out["batched_fp64_ms"] / out["batched_mixed_ms"]
    out["speedup_batched_mixed"] = out["plain_fp64_ms"] / out["batched_mixed_ms"]
    if params is not None:
        out["speedup_total"] = out["plain_fp64_ms"] / out["learned_batched_mixed_ms"]
        out["speedup_learned"] = out["batched_mixed_ms"] / out["learned_batched_mixed_ms"]
    # error of the mixed results against the FP64 ones on the GPU
    mu64, _ = ctx.bf_pcg_solve(sys_, 1e-10, precision=FP64)
    s64, _ = ctx.bf_diag_estimate(sys_, K, 0, 1e-10, precision=FP64)
    mu32, _ = ctx.bf_pcg_solve(sys_, tol, precision=MIXED)
    s32, _ = ctx.bf_diag_estimate(sys_, K, 0, tol, precision=MIXED)
    out["mixed_rel_err_vs_fp64"] = {"mean": float(torch.linalg.norm(mu32 - mu64) / torch.linalg.norm(mu64)),
                                    "variance": float(torch.linalg.norm(s32 - s64) / torch.linalg.norm(s64))}
    return out


def stream_copy_gbs():
    """Achieved device copy bandwidth (bytes read + written per second) of a
    plain 1 GiB copy: the practical HBM ceiling next to the 8 TB/s peak."""
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 2 * COPY_BYTES * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9


def _kernel_rooflines(tm, N, K, T, G, fp64):
    """Per-kernel HBM rooflines of the solver kernels in a timing table."""
    out = {}
    for kname, (launches, ms) in tm.items():
        if launches == 0:
            continue
        w = algorithmic_work(kname, N, K, T, G, 0, fp64=fp64,
                             estimate="block_verify" in tm and "hutch_final" not in tm)
        if w is None or w[2] != "hbm":
            continue
        gbs = w[0] / (ms * 1e-3 / launches) / 1e9
        out[kname] = {"launches": launches, "avg_us": 1e3 * ms / launches, "algorithmic_bytes_per_launch": w[0],
                      "achieved_GBps": gbs, "frac_of_8TBps": gbs / HBM_PEAK_GBS}
    return out


def solver_section(g, args):
    """The solver kernels where the working set far exceeds the 256 MB Infinity
    Cache: the full pass's scene and views on a 1024^3 grid of 1 mm voxels
    (several million band voxels) with a strong prior (lambda = 1e5, so that
    CG takes tens of iterations).  The mean PCG (one right-hand side) and the 64-probe block
    solve, each in mixed precision and FP64: iterations per second in the
    section 8(d) unit (voxel-iterations, voxel-column-iterations), the roofline
    of the iteration and of every solver kernel."""
    import torch
    import paper_2602_19697_amd as bf
    from synth import make_workload
    from synth.configs import regrid
    ctx, dev = g["ctx"], g["ctx"].device
    t0 = time.time()
    if args.solver_workload == "union1024" and g["wl"].name == "union512":
        wl = regrid(g["wl"], "union1024", 1024, 0.001)  # same depth maps: nothing to render
    else:
        wl = make_workload(args.solver_workload, device=dev)
    depth = torch.from_numpy(np.ascontiguousarray(wl.depth)).to(dev)
    poses = torch.from_numpy(np.ascontiguousarray(wl.poses)).to(dev)
    band = ctx.bf_build_band(bf.grid_struct(wl.G, wl.h, wl.origin, wl.tau, wl.band), wl.cam, depth, poses)
    lam, K, tol = 1e5, 64, 1e-6
    sys_ = ctx.bf_assemble(band, wl.cam, depth, poses, bf.noise_struct(*wl.noise), lam, wl.eps)
    N = band.n
    log(f"[solver] {wl.name}: N={N} built in {time.time() - t0:.1f}s")
    out = {"workload": wl.name, "band_voxels": N, "lambda": lam, "probes": K, "tol": tol,
           "float_block_vector_MB": N * K * 4 / 1e6}
    for prec, name in ((bf.L.BF_PREC_MIXED, "mixed"), (bf.L.BF_PREC_FP64, "fp64")):
        fp64 = name == "fp64"
        # mean: one right-hand side
        ctx.bf_pcg_solve(sys_, tol, precision=prec)  # warm-up (allocations)
        torch.cuda.synchronize()
        ctx.bf_get_timings()
        ctx.bf_set_timing(True)
        t0 = time.perf_counter()
        _, rep = ctx.bf_pcg_solve(sys_, tol, precision=prec)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ctx.bf_set_timing(False)
        tm = ctx.bf_get_timings()
        busy = sum(tm.get(k, (0, 0.0))[1] for k in ("pcg_A", "pcg_B"))
        per_unit = iteration_bytes(1, fp64)
        mean = {"iters": rep["iters"], "wall_ms": wall * 1e3, "voxel_iters_per_s": N * rep["iters"] / wall,
                "kernels": _kernel_rooflines(tm, N, 1, wl.T, wl.G, fp64)}
        if busy > 0:
            ach = N * rep["iters"] * per_unit / (busy * 1e-3) / 1e9
            mean["iteration_roofline"] = {"bytes_per_unit": per_unit, "busy_ms_A_B": busy, "achieved_GBps": ach,
                                          "frac_of_8TBps": ach / HBM_PEAK_GBS,
                                          "voxel_iters_per_s_in_A_B": N * rep["iters"] / (busy * 1e-3)}
        # the K-probe block solve
        ctx.bf_diag_estimate(sys_, K, 0, tol, precision=prec)  # warm-up (allocations)
        torch.cuda.synchronize()
        ctx.bf_get_timings()
        ctx.bf_set_timing(True)
        t0 = time.perf_counter()
        _, prep = ctx.bf_diag_estimate(sys_, K, 0, tol, precision=prec)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ctx.bf_set_timing(False)
        tm = ctx.bf_get_timings()
        kt = {k: {"total_ms": ms} for k, (launches, ms) in tm.items()}
        block = {"iters": prep["iters"], "column_iters": prep["col_iters"], "wall_ms": wall * 1e3,
                 "voxel_column_iters_per_s": N * prep["col_iters"] / wall,
                 "iteration_roofline": solver_roofline(kt, N, K, fp64, prep["col_iters"]),
                 "kernels": _kernel_rooflines(tm, N, K, wl.T, wl.G, fp64)}
        out[name] = {"mean": mean, "block": block}
        br = block["iteration_roofline"] or {}
        mr = mean.get("iteration_roofline", {})
        log(f"[solver] {wl.name} N={N} {name}: mean {rep['iters']} it {mean['wall_ms']:.1f} ms "
            f"({mr.get('achieved_GBps', 0):.0f} GB/s in A+B); block K={K} "
            f"{prep['iters']} it {block['wall_ms']:.1f} ms, {block['voxel_column_iters_per_s']:.3g} "
            f"voxel-column-iters/s ({br.get('achieved', 0):.0f} GB/s in A+B+verify)")
    # time to tolerance on this large system with 32 probes (learned start trained at lambda = 1e5)
    out["time_to_tol"] = compare_solvers(ctx, sys_, lam, 32, reps=2, plain_reps=1)
    t = out["time_to_tol"]
    log(f"[solver] time to 1e-6: plain {t['plain_fp64_ms']:.1f} ms, block fp64 {t['batched_fp64_ms']:.1f}, "
        f"block mixed {t['batched_mixed_ms']:.1f}, learned {t.get('learned_batched_mixed_ms', float('nan')):.1f}")
    sys_.free()
    band.free()
    return out


def trilinear_section(g, args):
    """Trilinear pixel-centric rows (eq. 4) on the step's workload: assembly
    time, mean solves (FP64 and mixed) and an 8-probe FP64 variance to 1e-6,
    and the HBM rate of the 27-point product pass (pcg_A).  Algorithmic bytes
    per row of that pass: nb26 (104 B) and the couplings (26 s), diag, p_old
    and z of the row in, p and q out (5 s), neighbour rows as cache hits."""
    import torch
    import paper_2602_19697_amd as bf
    ctx, wl = g["ctx"], g["wl"]
    S = int(round(wl.tau / wl.h))
    noise = bf.noise_struct(*wl.noise)
    band = ctx.bf_build_band(g["grid"], wl.cam, g["depth"], g["poses"])
    N = band.n

    def assemble():
        return ctx.bf_assemble_trilinear(band, wl.cam, g["depth"], g["poses"], noise, wl.lam, wl.eps, wl.lam_b,
                                         samples_per_side=S)
    assemble().free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        sys_ = assemble()
        sys_.free()
    torch.cuda.synchronize()
    asm_ms = 1e3 * (time.perf_counter() - t0) / 3
    sys_ = assemble()
    arr = sys_.arrays()
    out = {"workload": wl.name, "band_voxels": N, "samples_per_side": S, "samples": arr["n_samples"],
           "cells": arr["n_cells"], "assemble_ms": asm_ms, "tol": 1e-6}
    for prec, name in ((bf.L.BF_PREC_FP64, "fp64"), (bf.L.BF_PREC_MIXED, "mixed")):
        ctx.bf_pcg_solve(sys_, 1e-6, precision=prec)
        torch.cuda.synchronize()
        ctx.bf_get_timings()
        ctx.bf_set_timing(True)
        t0 = time.perf_counter()
        _, rep = ctx.bf_pcg_solve(sys_, 1e-6, precision=prec)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ctx.bf_set_timing(False)
        tm = ctx.bf_get_timings()
        s = 8 if name == "fp64" else 4
        launches, ms = tm.get("pcg_A", (0, 0.0))
        res = {"iters": rep["iters"], "refinements": rep["refinements"], "wall_ms": wall * 1e3,
               "voxel_pcg_iters_per_s": N * rep["iters"] / wall}
        if launches:
            amount = N * (104 + 26 * s + 5 * s)
            gbs = amount / (ms * 1e-3 / launches) / 1e9
            res["pcg_A"] = {"launches": launches, "avg_us": 1e3 * ms / launches,
                            "algorithmic_bytes_per_launch": amount, "achieved_GBps": gbs,
                            "frac_of_8TBps": gbs / HBM_PEAK_GBS}
        out[name] = res
    # FP64 probes: mixed probe solves on these systems do not converge (float
    # refinement cannot contract the Jacobi-scaled system)
    _, rep = ctx.bf_diag_estimate(sys_, 8, 0, 1e-6, precision=bf.L.BF_PREC_FP64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep = ctx.bf_diag_estimate(sys_, 8, 0, 1e-6, precision=bf.L.BF_PREC_FP64)
    torch.cuda.synchronize()
    out["variance_fp64_K8"] = {"iters": rep["iters"], "column_iters": rep["col_iters"],
                               "wall_ms": 1e3 * (time.perf_counter() - t0)}
    log(f"[trilinear] {wl.name}: {arr['n_samples']} samples in {arr['n_cells']} cells, assembly {asm_ms:.1f} ms; "
        f"mean fp64 {out['fp64']['iters']} it {out['fp64']['wall_ms']:.1f} ms, mixed {out['mixed']['iters']} it "
        f"{out['mixed']['wall_ms']:.1f} ms; 8-probe variance {rep['iters']} it {out['variance_fp64_K8']['wall_ms']:.1f} ms")
    sys_.free()
    band.free()
    return out


NN_OPS_PER_PAIR = 9  # 3 differences, 3 products, 2 sums, 1 minimum (FP64)


def postview_section(g, args, top=8):
    """The post-view utility of eq. (13) on the headline pass: the `top`
    candidates of the summed-variance walk are rescored with
    U = sum (s - s') over the band voxels with |mu| <= the band half-width,
    s' from the step's probes (same K, seed, precision and tolerance) once
    each candidate's view, predicted from mu at the sensor's 640x480, is fused
    as one more view; the probe solves start from s.  Times the rescoring."""
    import torch
    import paper_2602_19697_amd as bf
    ctx, wl = g["ctx"], g["wl"]
    prec = bf.L.BF_PREC_FP64 if args.precision == "fp64" else bf.L.BF_PREC_MIXED
    K = args.probes
    band = ctx.bf_build_band(g["grid"], wl.cam, g["depth"], g["poses"])
    sys_ = ctx.bf_assemble(band, wl.cam, g["depth"], g["poses"], g["noise"], wl.lam, wl.eps)
    x0 = lv = None
    if args.learned:
        params = torch.from_numpy(np.load(_weights(wl.lam))).to(ctx.device)
        x0, lv = ctx.bf_warm_start(sys_, params)
    mu, _ = ctx.bf_pcg_solve(sys_, args.tol, precision=prec, x0=x0)
    s, _ = ctx.bf_diag_estimate(sys_, K, 0, args.tol, precision=prec, logvar=lv)
    scores, best = ctx.bf_nbv_score(band, mu, s, g["cands"], wl.ray_cam)
    sc = scores.cpu().numpy()
    which = [int(i) for i in np.argsort(-sc, kind="stable")[:top]]

    def rescore():
        return ctx.bf_nbv_postview(sys_, mu, s, g["cands"], which, wl.cam, g["noise"], K, 0, args.tol, precision=prec,
                                   eps_band=wl.band, warm=True)

    rescore()  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U, pbest, _, reps = rescore()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.bf_get_timings()
    ctx.bf_set_timing(True)
    rescore()
    ctx.bf_set_timing(False)
    tm = ctx.bf_get_timings()
    sys_.free()
    band.free()
    log(f"[postview] top {top}: {dt * 1e3 / top:.2f} ms per candidate; walk best {best}, post-view best {pbest}")
    return {"workload": f"{wl.name}: the top {top} of {wl.n_cand} candidates by the summed-variance walk, rescored; "
                        f"{K} {args.precision} probes to {args.tol} from s; predicted views at "
                        f"{wl.cam.width}x{wl.cam.height}; Omega = band voxels with |mu| <= {wl.band} m",
            "candidates": which, "walk_scores": [int(sc[i]) for i in which], "postview_utility": U,
            "walk_best": int(best), "postview_best": int(pbest), "ms_per_candidate": dt * 1e3 / top,
            "probe_iters": [r["iters"] for r in reps], "used_warm_start": [r["used_warm_start"] for r in reps],
            "kernels_ms_per_candidate": {k: ms / top for k, (n, ms) in sorted(tm.items(), key=lambda kv: -kv[1][1])
                                         if ms / top > 0.005}}


def surface_section(g, args):
    """Algorithm 1 step 7 and the geometry metrics of Sec. 4.2 on the step's
    workload: marching-tetrahedra meshes of the coarse TSDF and of the mean of
    the voxel-centric system (without and with the boundary anchor) and of the
    trilinear system, each against 200k points of the analytic surface (F at
    5, 10, 20 mm).  Timings of extraction and of the all-pairs nearest-point
    kernel (ALU bound: 9 FP64 operations per pair)."""
    import torch
    import paper_2602_19697_amd as bf
    from synth import surface_points
    ctx, wl = g["ctx"], g["wl"]
    thr = (0.005, 0.01, 0.02)
    gt = torch.from_numpy(surface_points(wl.scene, 200000, 0)).to(ctx.device)
    noise = bf.noise_struct(*wl.noise)
    band = ctx.bf_build_band(g["grid"], wl.cam, g["depth"], g["poses"])
    fields = {"tsdf": band.arrays()["tsdf"]}
    for label, lam_b in (("mean", 0.0), ("mean_anchored", 10.0)):
        sys_ = ctx.bf_assemble(band, wl.cam, g["depth"], g["poses"], noise, wl.lam, wl.eps, lam_b)
        fields[label], _ = ctx.bf_pcg_solve(sys_, 1e-8, precision=bf.L.BF_PREC_FP64)
        sys_.free()
    S = int(round(wl.tau / wl.h))
    sys_ = ctx.bf_assemble_trilinear(band, wl.cam, g["depth"], g["poses"], noise, wl.lam, wl.eps,
                                     samples_per_side=S)
    fields["mean_trilinear"], _ = ctx.bf_pcg_solve(sys_, 1e-8, precision=bf.L.BF_PREC_FP64)
    sys_.free()
    out = {"gt_points": int(gt.shape[0]), "thresholds_m": list(thr), "meshes": {}}
    for label, field in fields.items():
        mesh = ctx.bf_extract_surface(band, field)
        v = mesh.arrays()["verts"]
        m = ctx.bf_surface_metrics(v, gt, thr)
        out["meshes"][label] = {"vertices": mesh.n_vert, "triangles": mesh.n_tri,
                                **{k: m[k] for k in ("chamfer", "accuracy", "completeness", "precision", "recall",
                                                     "fscore")}}
        mesh.free()
    # timings on the plain mean's mesh
    mesh_ms = _timed(lambda: ctx.bf_extract_surface(band, fields["mean"]).free(), reps=5)[1]
    mesh = ctx.bf_extract_surface(band, fields["mean"])
    v = mesh.arrays()["verts"]
    torch.cuda.synchronize()
    ctx.bf_get_timings()
    ctx.bf_set_timing(True)
    _, met_ms = _timed(lambda: ctx.bf_surface_metrics(v, gt, thr), reps=2)
    ctx.bf_set_timing(False)
    tm = ctx.bf_get_timings()
    launches, ms = tm.get("nn_dist2", (0, 0.0))
    pairs = 2 * mesh.n_vert * int(gt.shape[0])  # both directions
    out["extract_ms"] = mesh_ms
    out["metrics_ms"] = met_ms
    if launches:
        ach = pairs * NN_OPS_PER_PAIR / (ms * 1e-3 / launches * 2) / 1e12  # two launches per metrics call
        out["nn_dist2"] = {"launches": launches, "avg_us": 1e3 * ms / launches, "pairs_per_call": pairs,
                           "achieved_TOPs": ach, "peak_TOPs": FP64_ALU_PEAK_TOPS,
                           "frac": ach / FP64_ALU_PEAK_TOPS}
    mesh.free()
    band.free()
    mm = out["meshes"]
    log("[surface] " + "; ".join(f"{k}: CD {mm[k]['chamfer']:.2e} acc {1e3 * mm[k]['accuracy']:.2f} mm "
                                 f"comp {1e3 * mm[k]['completeness']:.2f} mm F@20 {mm[k]['fscore'][2]:.3f}"
                                 for k in mm) + f"; extract {mesh_ms:.2f} ms, metrics {met_ms:.1f} ms")
    return out


def batch_section(g, args):
    """Many scenes of uneven size: args.batch_scenes sphere scenes whose band
    sizes are log-uniform in [2e4, 8e5], mean + 64-probe variance, to 1e-6.
    The autotuner picks the schedule on the batch itself; then the batched
    mixed solve is timed against the same work done scene by scene in plain
    FP64 and batched in FP64."""
    import torch
    import paper_2602_19697_amd as bf
    from synth import make_workload
    ctx, dev = g["ctx"], g["ctx"].device
    FP64, MIXED = bf.L.BF_PREC_FP64, bf.L.BF_PREC_MIXED
    K, tol = args.batch_probes, 1e-6
    t0 = time.time()
    scenes = []
    for s in range(args.batch_scenes):
        wl = make_workload(f"batchsphere{s}", device=dev)
        depth = torch.from_numpy(np.ascontiguousarray(wl.depth)).to(dev)
        poses = torch.from_numpy(np.ascontiguousarray(wl.poses)).to(dev)
        band = ctx.bf_build_band(bf.grid_struct(wl.G, wl.h, wl.origin, wl.tau, wl.band), wl.cam, depth, poses)
        sys_ = ctx.bf_assemble(band, wl.cam, depth, poses, bf.noise_struct(*wl.noise), wl.lam, wl.eps)
        scenes.append((band, sys_))
    systems = [sy for _, sy in scenes]
    sizes = [b.n for b, _ in scenes]
    log(f"[batch] {len(scenes)} scenes, N total {sum(sizes)} (min {min(sizes)}, max {max(sizes)}) "
        f"built in {time.time() - t0:.1f}s")
    t0 = time.time()
    best, table = ctx.bf_autotune_batch(systems, K, 0, tol, precision=MIXED)
    log(f"[batch] autotuned over {len(table)} schedules in {time.time() - t0:.1f}s: {best.as_dict()}")
    mean_sched = bf.Context.schedule(best.rows_per_tile, best.blocks_per_cu, best.order, best.xcd_aware, 0)

    def batched(prec, sched_probe):
        def run():
            _, r = ctx.bf_pcg_solve_batched(systems, tol, precision=prec, schedule=mean_sched)
            _, pr = ctx.bf_diag_estimate_batched(systems, K, 0, tol, precision=prec, schedule=sched_probe)
            return sum(x["col_iters"] for x in r) + sum(x["col_iters"] for x in pr)
        return run

    def per_scene_plain():
        its = 0
        for sy in systems:
            _, r = ctx.bf_pcg_solve(sy, tol, precision=FP64)
            its += r["iters"]
            for k in range(K):
                _, pr = ctx.bf_diag_estimate(sy, 1, 1000 + k, tol, precision=FP64)
                its += pr["iters"]
        return its

    out = {"scenes": len(scenes), "band_voxels_total": int(sum(sizes)), "band_voxels_min": int(min(sizes)),
           "band_voxels_max": int(max(sizes)), "probes": K, "tol": tol, "schedule": best.as_dict(),
           "autotune_candidates": len(table)}
    for name, fn, reps in (("plain_fp64_per_scene", per_scene_plain, 1),
                           ("batched_fp64", batched(FP64, best), 3),
                           ("batched_mixed", batched(MIXED, best), 3)):
        its, ms = _timed(fn, reps)
        out[name + "_ms"] = ms
        out[name + "_column_iters"] = its
        log(f"[batch] {name}: {ms:.1f} ms")
    out["speedup_batched_mixed_vs_plain"] = out["plain_fp64_per_scene_ms"] / out["batched_mixed_ms"]
    # mixed vs FP64 on the GPU, worst scene
    m64, _ = ctx.bf_pcg_solve_batched(systems, 1e-10, precision=FP64, schedule=mean_sched)
    s64, _ = ctx.bf_diag_estimate_batched(systems, K, 0, 1e-10, precision=FP64, schedule=best)
    m32, _ = ctx.bf_pcg_solve_batched(systems, tol, precision=MIXED, schedule=mean_sched)
    s32, _ = ctx.bf_diag_estimate_batched(systems, K, 0, tol, precision=MIXED, schedule=best)
    rel = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    out["mixed_rel_err_vs_fp64_max"] = {"mean": max(rel(a, b) for a, b in zip(m32, m64)),
                                        "variance": max(rel(a, b) for a, b in zip(s32, s64))}
    # error against the FP64 oracle (its own band, FP64 PCG to 1e-10, the same
    # seeded probes) on the smallest, two middle and the largest scene
    if not args.no_cpu_baseline:
        import oracle as O
        by_size = sorted(range(len(scenes)), key=lambda i: sizes[i])
        pick = sorted({by_size[0], by_size[len(by_size) // 3], by_size[2 * len(by_size) // 3], by_size[-1]})
        errs = []
        t0 = time.time()
        for i in pick:
            wl = make_workload(f"batchsphere{i}")
            ref = O.full_pipeline(wl)
            mu = O.pcg(ref["nbr"], ref["diag"], wl.lam, ref["rhs"], 1e-10)[0]
            sv = O.hutchinson(ref["nbr"], ref["diag"], wl.lam, K, 0, 1e-10)
            np_rel = lambda a, b: float(np.linalg.norm(a.cpu().numpy() - b) / np.linalg.norm(b))
            errs.append({"scene": i, "band_voxels": sizes[i], "band_equal": bool(len(ref["keys"]) == sizes[i]),
                         "mixed_mean": np_rel(m32[i], mu), "mixed_variance": np_rel(s32[i], sv),
                         "fp64_mean": np_rel(m64[i], mu), "fp64_variance": np_rel(s64[i], sv)})
        out["rel_err_vs_fp64_oracle"] = errs
        log(f"[batch] vs FP64 oracle ({time.time() - t0:.1f} s): " + "; ".join(
            f"scene {e['scene']} N={e['band_voxels']} mixed {e['mixed_mean']:.1e}/{e['mixed_variance']:.1e}"
            for e in errs))
    for band, sy in scenes:
        sy.free()
        band.free()
    return out


def _oracle_stages(O, wl, og, oc, depth, poses, keys, nbr, deg, args, rng):
    """Seconds of each oracle stage on the bounded sample, extrapolated to one
    whole step of the timed configuration."""
    N = len(keys)
    t = {}
    # TSDF: a random voxel sample of the grid, every view per voxel
    ns = args.cpu_tsdf_sample
    idx = rng.integers(0, wl.G, size=(ns, 3)).astype(np.int32)
    t0 = time.perf_counter()
    O.tsdf_points(og, oc, depth, poses, idx)
    t["tsdf"] = (time.perf_counter() - t0) / ns * wl.G ** 3
    # assembly on a sample of band voxels
    na = min(N, args.cpu_assembly_sample)
    sel = np.sort(rng.choice(N, size=na, replace=False))
    t0 = time.perf_counter()
    O.assemble(og, oc, depth, poses, keys[sel], noise=wl.noise)
    t["assembly"] = (time.perf_counter() - t0) / na * N
    Lam, b = O.assemble(og, oc, depth, poses, keys, noise=wl.noise)
    diag = O.precision_diag(Lam, deg, wl.lam, wl.eps)
    # the whole mean solve
    t0 = time.perf_counter()
    mu, rep = O.pcg(nbr, diag, wl.lam, b, args.tol)
    t["pcg"] = time.perf_counter() - t0
    # probe solves: a few, extrapolated to K
    kp = min(args.probes, args.cpu_probe_sample)
    t0 = time.perf_counter()
    s, its = O.hutchinson(nbr, diag, wl.lam, kp, 0, args.tol, with_iters=True)
    t["probes"] = (time.perf_counter() - t0) / kp * args.probes
    # NBV: a few candidates, extrapolated to all
    q = O.quantize_variance(s)
    cands = wl.candidates()
    nc = args.cpu_nbv_sample
    t0 = time.perf_counter()
    O.nbv_scores(og, O.cam(wl.ray_cam), keys, mu, q, cands, which=list(range(0, len(cands), len(cands) // nc))[:nc])
    t["nbv"] = (time.perf_counter() - t0) / nc * len(cands)
    work = N * (rep["iters"] + int(np.mean(its)) * args.probes)
    return t, work, dict(ns=ns, na=na, kp=kp, nc=nc, N=N, ncand=len(cands))


def cpu_baseline(g, args):
    """The FP64 oracle, as it stands, on a bounded sample of the timed step's
    workload, extrapolated to one whole step and expressed in
    voxel-PCG-iterations/s: once on one thread and once on every host core its
    OpenMP loops may use (voxels, probes and candidates in parallel; the mean
    PCG is serial).  The oracle builds its own band first (untimed)."""
    import oracle as O
    wl = g["wl"]
    og = O.grid_of(wl)
    oc = O.cam(wl.cam)
    depth = np.ascontiguousarray(wl.depth)
    poses = np.ascontiguousarray(wl.poses)
    cores = O.max_threads()
    t0 = time.time()
    td, wd = O.tsdf_dense(og, oc, depth, poses)
    keys, bt, bw = O.band(og, td, wd)
    del td, wd
    nbr, deg = O.neighbours(wl.G, keys)
    log(f"[cpu] oracle band N={len(keys)} prepared in {time.time() - t0:.1f}s on {cores} threads")
    runs = {}
    for n in (1, cores):
        O.set_threads(n)
        t, work, smp = _oracle_stages(O, wl, og, oc, depth, poses, keys, nbr, deg, args, np.random.default_rng(0))
        runs[n] = (t, work)
        log(f"[cpu] {n} thread(s): extrapolated step {sum(t.values()):.1f} s " +
            ", ".join(f"{k} {v:.2f}" for k, v in t.items()))
    O.set_threads(cores)
    t1, work = runs[1]
    tn, _ = runs[cores]
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"value": work / sum(tn.values()), "unit": "voxel-PCG-iters/s", "cores": cores, "kind": "oracle",
            "sample": (f"FP64 oracle on {cores} threads: TSDF of {smp['ns']} random voxels x {wl.T} views, "
                       f"assembly of {smp['na']} band voxels, the full mean PCG (N={smp['N']}), {smp['kp']} of "
                       f"{args.probes} probe solves and NBV of {smp['nc']} of {smp['ncand']} candidates, each "
                       f"extrapolated to the whole step; the same sample on one thread is single_thread"),
            "extrapolated_step_s": sum(tn.values()), "stage_s": tn,
            "single_thread": {"value": work / sum(t1.values()), "cores": 1, "extrapolated_step_s": sum(t1.values()),
                              "stage_s": t1},
            "host": {"omp_threads": cores, "os_cpu_count": os.cpu_count(), "affinity_cpus": affinity}}


def _scene_words(wl):
    from collections import Counter
    kinds = Counter(type(p).__name__ for p in getattr(wl.scene, "prims", []))
    names = {"Sphere": "spheres", "RoundedBox": "rounded boxes", "Torus": "tori"}
    return "union of " + ", ".join(f"{n} {names.get(k, k)}" for k, n in kinds.items())


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    # 20 timed steps (under 0.1 s): the 2 with per-kernel event timing, which
    # costs host time at every launch, then weigh 10% of the average
    ap.add_argument("--steps", type=int, default=20)
    # the first process on a box ran its first timed steps with 2 ms/step more
    # host idle (the same kernels): warm up longer
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--timing-steps", type=int, default=2,
                    help="per-kernel HIP event timing on the last this many timed steps")
    ap.add_argument("--workload", default="union512")
    ap.add_argument("--probes", type=int, default=32)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="mixed",
                    help="solver precision of the timed step (the 512^3 full pass is mixed)")
    ap.add_argument("--no-learned", dest="learned", action="store_false",
                    help="start the timed solves from zero instead of the learned network")
    ap.add_argument("--section-workload", default="union256",
                    help="workload of the FP64 step section and of the trilinear and surface sections")
    ap.add_argument("--no-section-step", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-solver-roofline", action="store_true")
    ap.add_argument("--no-trilinear", action="store_true")
    ap.add_argument("--no-surface", action="store_true")
    ap.add_argument("--no-postview", action="store_true")
    ap.add_argument("--allocator", choices=("pool", "torch"), default="torch",
                    help="where bands and systems get their memory: the library's pool or torch's allocator")
    ap.add_argument("--solver-workload", default="union1024")
    ap.add_argument("--batch-scenes", type=int, default=32)
    ap.add_argument("--batch-probes", type=int, default=64)
    ap.add_argument("--cpu-tsdf-sample", type=int, default=1000000)
    ap.add_argument("--cpu-assembly-sample", type=int, default=400000)
    ap.add_argument("--cpu-probe-sample", type=int, default=4)
    ap.add_argument("--cpu-nbv-sample", type=int, default=8)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the narrow-band solve runs on a single MI355X "
              "(see DESIGN.md for how it would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    g = run_gpu(args)
    log(f"[bench] {g['wl'].name}: {g['ms_step']:.3f} ms/step, {g['value']:.4g} voxel-PCG-iters/s")
    # the 256^3 FP64 step (no learned start), and the sections that run on it
    g2 = None
    if not args.no_section_step or not args.no_trilinear or not args.no_surface:
        a2 = argparse.Namespace(**{**vars(args), "workload": args.section_workload, "precision": "fp64",
                                   "learned": False, "warmup": 2})
        g2 = run_gpu(a2)
        log(f"[bench] {g2['wl'].name} FP64: {g2['ms_step']:.3f} ms/step")
    cmp = None if args.no_compare else time_to_tol(g, args)
    sweep = None
    if not args.no_compare:
        sweep = [time_to_tol(g, args, lam) for lam in (1e3, 1e5)]
    solver = None if args.no_solver_roofline else solver_section(g, args)
    copy_gbs = None if args.no_compare else stream_copy_gbs()
    batch = None if args.no_batch else batch_section(g, args)
    trilinear = None if args.no_trilinear else trilinear_section(g2, args)
    surface = None if args.no_surface else surface_section(g2, args)
    postview = None if args.no_postview else postview_section(g, args)
    cpu = None if args.no_cpu_baseline else cpu_baseline(g, args)
    wl = g["wl"]
    roof = g["solver_roofline"]
    if roof is not None:
        # HBM bytes of the same launches (every launch the roofline times), from
        # the committed counters of each kernel
        per = [(measured_traffic(k, wl.name), g["kernels"][k]["launches"]) for k in SOLVER_ITERATION
               if k in g["kernels"]]
        traffic = None if not per or any(t is None for t, _ in per) else sum(t * n for t, n in per)
        roof = dict(roof, traffic=traffic,
                    traffic_per_unit=None if traffic is None else traffic / roof["units"])
    top = g["dominant"]
    nbv = g["kernels"].get("nbv_rays")
    rays = wl.n_cand * wl.ray_cam.width * wl.ray_cam.height
    steps = g["info"]["walk_steps"]
    nbv_info = None if nbv is None else {
        "rays_per_launch": rays, "avg_ms": nbv["avg_us"] * 1e-3, "rays_per_s": rays / (nbv["avg_us"] * 1e-6),
        "dda_steps_per_launch": steps, "dda_steps_per_s": steps / (nbv["avg_us"] * 1e-6),
        "share_of_step": nbv["share_of_step"], "bound": "latency / instruction issue (no roofline claim)"}
    section_step = None
    if g2 is not None and not args.no_section_step:
        w2 = g2["wl"]
        section_step = {
            "workload": f"{w2.name}: {_scene_words(w2)}; {w2.G}^3 grid, h={w2.h} m, {w2.T} views "
                        f"{w2.cam.width}x{w2.cam.height}; FP64 PCG tol {args.tol} from zero, {args.probes}-probe "
                        f"FP64 block PCG, NBV 512x160x120",
            "ms_per_step": g2["ms_step"], "voxel_pcg_iters_per_s": g2["value"], "band_voxels": g2["info"]["N"],
            "pcg_iters": g2["info"]["iters"], "probe_iters": g2["info"]["probe_iters"],
            "solver_roofline": g2["solver_roofline"], "rooflines": g2["rooflines"], "kernels": g2["kernels"]}
    line = {
        "metric": "band voxel-PCG-iters/s, probe-solves/s; learned+batched vs plain time-to-1e-6",
        "value": g["value"],
        "unit": "voxel-PCG-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": g["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name} full pass: {_scene_words(wl)}; {wl.G}^3 grid, "
                               f"h={wl.h} m, band +-{round(wl.band / wl.h)} voxels, {wl.T} views "
                               f"{wl.cam.width}x{wl.cam.height}; {args.precision.upper()} PCG tol {args.tol}"
                               f"{' from the learned start' if args.learned else ''}, "
                               f"{args.probes}-probe {args.precision.upper()} block PCG"
                               f"{' from the learned log-variance' if args.learned else ''}, NBV 512x160x120",
                   "band_voxels": g["info"]["N"], "pcg_iters": g["info"]["iters"],
                   "probe_iters": g["info"]["probe_iters"], "parallelism": "single GPU"},
        "probe_solves_per_s": args.probes / (g["ms_step"] * 1e-3),
        "roofline": roof,
        "largest_kernel": {"name": top, "share_of_step": g["kernels"][top]["share_of_step"]} if top else None,
        "nbv": nbv_info,
        "rooflines": g["rooflines"],
        "kernels": g["kernels"],
        "step_fp64_union256": section_step,
        "time_to_tol": cmp,
        "time_to_tol_lambda_sweep": sweep,
        "solver_rooflines_sized": solver,
        "stream_copy_GBps": copy_gbs,
        "batch": batch,
        "trilinear": trilinear,
        "surface": surface,
        "nbv_postview": postview,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
