#!/usr/bin/env python3
"""Throughput of the narrow-band Bayesian SDF solve on one MI355X.

One step is one pass of the whole hot path over the 256^3 union scene (3
spheres, a rounded box and a torus; 4 mm voxels, +-4 voxel band, 40 views at
640x480 on a 1.2 m hemisphere, sigma(z) depth noise):
  coarse TSDF + band + hash + neighbours  ->  assembly of Lambda, b, diag(Q)
  ->  FP64 Jacobi-PCG for the mean (tol 1e-6)  ->  32-probe Hutchinson
  variance as one FP64 block-PCG (tol 1e-6)  ->  NBV scoring of 512 candidate
  poses (160x120 rays each) with argmax.
Inputs are synthetic and resident in device memory before timing starts.

Printed: one JSON line with the metric (band voxel-PCG-iterations per second
of step time), the dominant kernel's roofline (algorithmic bytes or flops per
launch over its event-timed average duration), the learned/batched/mixed vs
plain FP64 time-to-tolerance comparison, and the FP64 CPU oracle timed on a
bounded sample of the same workload.
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


def algorithmic_work(name, N, K, T, G, P, fp64=True):
    """(amount, unit, bound) of one launch of a timed kernel."""
    s = 8 if fp64 else 4
    if name == "pcg_A":      # nbr, diag, z, p_old -> p_new, q
        return N * (24 + 5 * s), "B", "hbm"
    if name == "pcg_B":      # dinv, p, q, x, r -> x, r, z
        return N * 8 * s, "B", "hbm"
    if name == "block_A":    # nbr, diag; per column zz, p_old -> p_new, q
        return N * (24 + s + 4 * K * s), "B", "hbm"
    if name == "block_B":    # dinv; per column p, q, x, r -> x, r, zz
        return N * (s + 8 * K * s), "B", "hbm"
    if name == "tsdf_count":  # 35 FP64 operations per voxel and view + dense store
        return G ** 3 * T * 35, "flop", "alu"
    if name == "assemble":
        return N * T * 45, "flop", "alu"
    return None


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
    ctx = bf.Context(dev)
    K = args.probes

    def step():
        band = ctx.bf_build_band(grid, wl.cam, depth, poses)
        sys_ = ctx.bf_assemble(band, wl.cam, depth, poses, noise, wl.lam, wl.eps)
        mu, rep = ctx.bf_pcg_solve(sys_, args.tol, precision=bf.L.BF_PREC_FP64)
        s, prep = ctx.bf_diag_estimate(sys_, K, 0, args.tol, precision=bf.L.BF_PREC_FP64)
        scores, best = ctx.bf_nbv_score(band, mu, s, cands, wl.ray_cam)
        out = dict(N=band.n, iters=rep["iters"], probe_iters=prep["iters"],
                   work=band.n * (rep["col_iters"] + prep["col_iters"]), best=best,
                   rel_res=rep["rel_res"], probe_rel_res=prep["rel_res"])
        sys_.free()
        band.free()
        return out

    for _ in range(args.warmup):
        info = step()
    torch.cuda.synchronize()
    ctx.bf_set_timing(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    works = []
    for _ in range(args.steps):
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

    # kernel table and the dominant kernel's roofline
    kernels = {}
    for name, (launches, ms) in sorted(timings.items(), key=lambda kv: -kv[1][1]):
        kernels[name] = {"launches": launches, "avg_us": 1e3 * ms / max(launches, 1),
                         "share_of_step": ms / args.steps / ms_step}
    P = 1
    while P < wl.G:
        P *= 2
    rooflines = {}
    for name, kt in kernels.items():
        w = algorithmic_work(name, info["N"], K, wl.T, wl.G, P)
        if w is None:
            continue
        amount, unit, bound = w
        avg_s = kt["avg_us"] * 1e-6
        if unit == "B":
            ach = amount / avg_s / 1e9
            rooflines[name] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": ach / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": amount}
        else:
            ach = amount / avg_s / 1e12
            rooflines[name] = {"bound": "alu", "achieved": ach, "peak": FP64_ALU_PEAK_TOPS,
                               "unit": "TFLOP/s", "frac": ach / FP64_ALU_PEAK_TOPS,
                               "algorithmic_flops_per_launch": amount}
    dominant = next(iter(kernels)) if kernels else None
    return dict(ctx=ctx, wl=wl, depth=depth, poses=poses, cands=cands, grid=grid, noise=noise,
                info=info, value=value, ms_step=ms_step, kernels=kernels, rooflines=rooflines,
                dominant=dominant)


def time_to_tol(g, args):
    """Plain FP64 (mean + K sequential probe solves from zero) vs one mixed
    mean solve + one mixed K-column block solve."""
    import torch
    import paper_2602_19697_amd as bf
    ctx, wl = g["ctx"], g["wl"]
    band = ctx.bf_build_band(g["grid"], wl.cam, g["depth"], g["poses"])
    sys_ = ctx.bf_assemble(band, wl.cam, g["depth"], g["poses"], g["noise"], wl.lam, wl.eps)
    K, tol = args.probes, 1e-6

    def plain():
        _, r = ctx.bf_pcg_solve(sys_, tol, precision=bf.L.BF_PREC_FP64)
        its = r["iters"]
        for k in range(K):
            _, pr = ctx.bf_diag_estimate(sys_, 1, 1000 + k, tol, precision=bf.L.BF_PREC_FP64)
            its += pr["iters"]
        return its

    def batched_mixed():
        _, r = ctx.bf_pcg_solve(sys_, tol, precision=bf.L.BF_PREC_MIXED)
        _, pr = ctx.bf_diag_estimate(sys_, K, 0, tol, precision=bf.L.BF_PREC_MIXED)
        return r["iters"] + pr["iters"]

    def batched_fp64():
        _, r = ctx.bf_pcg_solve(sys_, tol, precision=bf.L.BF_PREC_FP64)
        _, pr = ctx.bf_diag_estimate(sys_, K, 0, tol, precision=bf.L.BF_PREC_FP64)
        return r["iters"] + pr["iters"]

    out = {}
    for name, fn in (("plain_fp64", plain), ("batched_fp64", batched_fp64), ("batched_mixed", batched_mixed)):
        fn()
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            its = fn()
        torch.cuda.synchronize()
        out[name + "_ms"] = 1e3 * (time.perf_counter() - t0) / reps
    out["speedup_batching"] = out["plain_fp64_ms"] / out["batched_fp64_ms"]
    out["speedup_precision"] = out["batched_fp64_ms"] / out["batched_mixed_ms"]
    out["speedup_total"] = out["plain_fp64_ms"] / out["batched_mixed_ms"]
    out["learned"] = None
    sys_.free()
    band.free()
    return out


def cpu_baseline(g, args):
    """FP64 oracle on a bounded sample of the same workload, single thread,
    extrapolated to one whole step and expressed in voxel-PCG-iterations/s."""
    import oracle as O
    wl = g["wl"]
    og = O.grid_of(wl)
    oc = O.cam(wl.cam)
    rng = np.random.default_rng(0)
    depth = np.ascontiguousarray(wl.depth)
    poses = np.ascontiguousarray(wl.poses)
    # untimed preparation: the oracle's own band (dense TSDF uses OpenMP here)
    t0 = time.time()
    td, wd = O.tsdf_dense(og, oc, depth, poses)
    keys, bt, bw = O.band(og, td, wd)
    nbr, deg = O.neighbours(wl.G, keys)
    log(f"[cpu] oracle band N={len(keys)} prepared in {time.time() - t0:.1f}s")
    N = len(keys)
    t = {}
    # TSDF: per-voxel cost on a random voxel sample
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
    # full mean solve
    t0 = time.perf_counter()
    mu, rep = O.pcg(nbr, diag, wl.lam, b, args.tol)
    t["pcg"] = time.perf_counter() - t0
    # probe solves: a few, extrapolated to K
    kp = min(args.probes, args.cpu_probe_sample)
    t0 = time.perf_counter()
    s, its = O.hutchinson(nbr, diag, wl.lam, kp, 0, args.tol, with_iters=True)
    t["probes"] = (time.perf_counter() - t0) / kp * args.probes
    # NBV: one candidate, extrapolated to all
    q = O.quantize_variance(s)
    cands = wl.candidates()
    t0 = time.perf_counter()
    O.nbv_scores(og, O.cam(wl.ray_cam), keys, mu, q, cands, which=[0])
    t["nbv"] = (time.perf_counter() - t0) * len(cands)
    t_step = sum(t.values())
    work = N * (rep["iters"] + int(np.mean(its)) * args.probes)
    return {"value": work / t_step, "unit": "voxel-PCG-iters/s", "cores": 1, "kind": "oracle",
            "sample": (f"single-thread FP64 oracle: TSDF of {ns} random voxels x {wl.T} views, assembly of "
                       f"{na} band voxels, the full mean PCG (N={N}), {kp} of {args.probes} probe solves "
                       f"and NBV of 1 of {len(cands)} candidates, each extrapolated to the whole step"),
            "extrapolated_step_s": t_step, "stage_s": t}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="union256")
    ap.add_argument("--probes", type=int, default=32)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--cpu-tsdf-sample", type=int, default=200000)
    ap.add_argument("--cpu-assembly-sample", type=int, default=40000)
    ap.add_argument("--cpu-probe-sample", type=int, default=2)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the narrow-band solve runs on a single MI355X "
              "(see DESIGN.md for how it would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    g = run_gpu(args)
    cmp = None if args.no_compare else time_to_tol(g, args)
    cpu = None if args.no_cpu_baseline else cpu_baseline(g, args)
    dom = g["dominant"]
    roof = g["rooflines"].get(dom)
    if roof is None and g["rooflines"]:
        dom = max(g["rooflines"], key=lambda k: g["kernels"][k]["share_of_step"])
        roof = g["rooflines"][dom]
    if roof is not None:
        roof = dict(roof, kernel=dom, traffic=None)
    wl = g["wl"]
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: union of 3 spheres, rounded box, torus; {wl.G}^3 grid, "
                               f"h={wl.h} m, band +-{round(wl.band / wl.h)} voxels, {wl.T} views "
                               f"{wl.cam.width}x{wl.cam.height}; FP64 PCG tol {args.tol}, "
                               f"{args.probes}-probe block PCG, NBV 512x160x120",
                   "band_voxels": g["info"]["N"], "pcg_iters": g["info"]["iters"],
                   "probe_iters": g["info"]["probe_iters"], "parallelism": "single GPU"},
        "probe_solves_per_s": args.probes / (g["ms_step"] * 1e-3),
        "roofline": roof,
        "rooflines": g["rooflines"],
        "kernels": g["kernels"],
        "time_to_tol": cmp,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
