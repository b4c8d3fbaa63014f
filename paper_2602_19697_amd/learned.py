"""Training and evaluation of the learned warm start.

The network (libbf.so: bf_features, bf_mlp_forward, bf_warm_start,
bf_mlp_grad, bf_adam_step) learns, per band voxel, the correction of the
posterior mean to the Jacobi estimate rhs/diag (in voxel units) and the log of
the variance relative to 1/diag.  Training pairs come from the method's own
solves: the FP64 PCG mean (tol 1e-10) and a 64-probe FP64 Hutchinson estimate
of every training scene.  The solvers always run to their tolerance from the
proposed start, so the network can only change how many iterations they take.

    python -m paper_2602_19697_amd.learned --lam 10 --out weights.npy [--checkpoint ck.npz [--resume]]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import L, Context, grid_struct, noise_struct

N_TRAIN = L.BF_MLP_TRAIN
N_PARAMS = L.BF_MLP_PARAMS
WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
_WEIGHT_NAMES = {10.0: "warm_start_lam10", 1e5: "warm_start_lam1e5"}


def weights_path(lam: float, report: bool = False) -> str:
    """The committed network (or its training report) for prior strength lam."""
    if float(lam) not in _WEIGHT_NAMES:
        raise KeyError(f"no trained warm start for lambda={lam}; trained: {sorted(_WEIGHT_NAMES)}")
    return os.path.join(WEIGHTS_DIR, _WEIGHT_NAMES[float(lam)] + (".json" if report else ".npy"))
_SHAPES = [(64, 12), (64,), (64, 64), (64,), (64, 64), (64,), (2, 64), (2,)]


def init_params(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases, identity input/output scaling."""
    rng = np.random.default_rng(seed)
    parts = []
    for shp in _SHAPES:
        if len(shp) == 2:
            lim = math.sqrt(6.0 / (shp[0] + shp[1]))
            parts.append(rng.uniform(-lim, lim, size=shp).ravel())
        else:
            parts.append(np.zeros(shp))
    parts += [np.zeros(12), np.ones(12), np.zeros(2), np.ones(2)]
    return np.concatenate(parts).astype(np.float32)


def zero_params() -> np.ndarray:
    """A network whose outputs are exactly 0: x0 = rhs/diag, logvar = 0."""
    p = np.zeros(N_PARAMS, dtype=np.float32)
    p[N_TRAIN + 12:N_TRAIN + 24] = 1.0  # in_std
    p[N_TRAIN + 26:N_TRAIN + 28] = 1.0  # out_std
    return p


def set_scaling(params: np.ndarray, feat: np.ndarray, tgt: np.ndarray) -> np.ndarray:
    p = params.copy()
    p[N_TRAIN:N_TRAIN + 12] = feat.mean(0)
    p[N_TRAIN + 12:N_TRAIN + 24] = feat.std(0) + 1e-6
    p[N_TRAIN + 24:N_TRAIN + 26] = tgt.mean(0)
    p[N_TRAIN + 26:N_TRAIN + 28] = tgt.std(0) + 1e-12
    return p


def scene_system(ctx: Context, wl, lam: float):
    dev = ctx.device
    depth = torch.from_numpy(np.ascontiguousarray(wl.depth)).to(dev)
    poses = torch.from_numpy(np.ascontiguousarray(wl.poses)).to(dev)
    band = ctx.bf_build_band(grid_struct(wl.G, wl.h, wl.origin, wl.tau, wl.band), wl.cam, depth, poses)
    sys_ = ctx.bf_assemble(band, wl.cam, depth, poses, noise_struct(*wl.noise), lam, wl.eps)
    return band, sys_


def scene_pairs(ctx: Context, wl, lam: float, probes: int = 64, seed: int = 0):
    """Features [N][12] (device) and targets [N][2] (host) of one scene: the
    FP64 mean (tol 1e-10) and a `probes`-probe FP64 Hutchinson estimate, turned
    into targets by the library (bf_warm_start_targets)."""
    band, sys_ = scene_system(ctx, wl, lam)
    feat = ctx.bf_features(sys_)
    mu, _ = ctx.bf_pcg_solve(sys_, 1e-10, precision=L.BF_PREC_FP64)
    s, _ = ctx.bf_diag_estimate(sys_, probes, seed, 1e-8, precision=L.BF_PREC_FP64)
    tgt = ctx.bf_warm_start_targets(sys_, mu, s).cpu().numpy()
    sys_.free()
    band.free()
    return feat, tgt


def training_scenes(n_sphere: int = 100, n_union: int = 70, n_union256: int = 30):
    """The training scenes: seeded spheres (voxel edge 12-20 mm), 128^3 unions
    (8 mm) and 256^3 unions (4 mm), all with seeds disjoint from the held-out ones."""
    return ([f"trainsphere{s}" for s in range(n_sphere)] + [("union128", 100 + s) for s in range(n_union)]
            + [("union256", 100 + s) for s in range(n_union256)])


def save_checkpoint(path: str, params, m, v, step: int, rng: np.random.Generator, hist) -> None:
    """Everything a resumed run needs to continue bit for bit: the FP32
    parameters, Adam's moments, the step and the minibatch generator's state."""
    tmp = path + ".tmp.npz"
    np.savez(tmp, params=params.cpu().numpy(), m=m.cpu().numpy(), v=v.cpu().numpy(), step=np.int64(step),
             rng=np.frombuffer(json.dumps(rng.bit_generator.state).encode(), dtype=np.uint8),
             hist=np.asarray(hist, dtype=np.float64).reshape(-1, 2))
    os.replace(tmp, path)


def load_checkpoint(path: str):
    with np.load(path, allow_pickle=False) as z:
        state = json.loads(bytes(z["rng"]).decode())
        return (z["params"], z["m"], z["v"], int(z["step"]), state,
                [(int(a), float(b)) for a, b in z["hist"]])


def train(ctx: Context, feats, tgts_host, steps: int = 3000, batch: int = 16384, lr: float = 2e-3,
          seed: int = 0, log_every: int = 500, checkpoint: str = None, checkpoint_every: int = 500,
          resume: bool = False, stop_at: int = None):
    """Adam on minibatches drawn with replacement; returns the FP32 parameters.
    With `checkpoint`, the state is saved every `checkpoint_every` steps and at
    the end; with `resume`, training continues from that file (same results as
    an uninterrupted run).  stop_at ends the run early after that step (an
    interrupted run, to be resumed with the same `steps`)."""
    dev = ctx.device
    feat_host = feats.cpu().numpy()
    params = torch.from_numpy(set_scaling(init_params(seed), feat_host, tgts_host)).to(dev)
    tgts = torch.from_numpy(tgts_host).to(dev)
    m = torch.zeros(N_TRAIN, dtype=torch.float32, device=dev)
    v = torch.zeros(N_TRAIN, dtype=torch.float32, device=dev)
    grad = torch.empty(N_TRAIN, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed)
    n = feats.shape[0]
    hist = []
    start = 1
    if resume and checkpoint and os.path.exists(checkpoint):
        p0, m0, v0, done, state, hist = load_checkpoint(checkpoint)
        params = torch.from_numpy(p0).to(dev)
        m = torch.from_numpy(m0).to(dev)
        v = torch.from_numpy(v0).to(dev)
        rng.bit_generator.state = state
        start = done + 1
        print(f"[train] resumed at step {done} from {checkpoint}", file=sys.stderr, flush=True)
    for step in range(start, steps + 1):
        idx = torch.from_numpy(rng.integers(0, n, size=batch).astype(np.int32)).to(dev)
        ctx.bf_mlp_grad(params, feats, tgts, idx, grad, loss)
        rate = lr * 0.5 * (1.0 + math.cos(math.pi * step / steps))  # cosine decay
        ctx.bf_adam_step(params, m, v, grad, step, lr=rate)
        if step % log_every == 0 or step == 1:
            hist.append((step, float(loss.item())))
            print(f"[train] step {step} loss {hist[-1][1]:.4f}", file=sys.stderr, flush=True)
        if checkpoint and (step % checkpoint_every == 0 or step == steps):
            save_checkpoint(checkpoint, params, m, v, step, rng, hist)
        if stop_at is not None and step >= stop_at:
            break
    return params.cpu().numpy(), hist


def evaluate(ctx: Context, wl, lam: float, params: np.ndarray, tol: float = 1e-6, probes: int = 32,
             precision=L.BF_PREC_FP64, reps: int = 3):
    """Iterations and time to tol from x0 = 0, the Jacobi start and the learned
    start, probe iterations with and without the learned log-variance, and the
    learned outputs' errors against the FP64 solves."""
    band, sys_ = scene_system(ctx, wl, lam)
    dev = ctx.device
    feat = ctx.bf_features(sys_)
    p_learn = torch.from_numpy(params).to(dev)
    p_zero = torch.from_numpy(zero_params()).to(dev)
    out = {"N": band.n, "lam": lam}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return r, 1e3 * (time.perf_counter() - t0) / reps

    mu_ref, _ = ctx.bf_pcg_solve(sys_, 1e-10, precision=L.BF_PREC_FP64)
    s_ref, _ = ctx.bf_diag_estimate(sys_, 64, 777, 1e-8, precision=L.BF_PREC_FP64)
    mu_ref_h = mu_ref.cpu().numpy()
    nrm = np.linalg.norm(mu_ref_h)
    (_, r0), t_zero = timed(lambda: ctx.bf_pcg_solve(sys_, tol, precision=precision))
    (_, rj), t_jac = timed(lambda: ctx.bf_pcg_solve(sys_, tol, precision=precision,
                                                    x0=ctx.bf_warm_start(sys_, p_zero, feat, logvar=False)[0]))

    def learned_mean():  # features + network + solve
        f = ctx.bf_features(sys_)
        x0, _ = ctx.bf_warm_start(sys_, p_learn, f, logvar=False)
        return ctx.bf_pcg_solve(sys_, tol, precision=precision, x0=x0)
    (_, rl), t_learn = timed(learned_mean)
    x0_j, _ = ctx.bf_warm_start(sys_, p_zero, feat, logvar=False)
    x0_l, lv = ctx.bf_warm_start(sys_, p_learn, feat)
    out["mean"] = {
        "iters_zero": r0["iters"], "iters_jacobi": rj["iters"], "iters_learned": rl["iters"],
        "ms_zero": t_zero, "ms_jacobi": t_jac, "ms_learned_incl_features_mlp": t_learn,
        "start_err_jacobi": float(np.linalg.norm(x0_j.cpu().numpy() - mu_ref_h) / nrm),
        "start_err_learned": float(np.linalg.norm(x0_l.cpu().numpy() - mu_ref_h) / nrm)}
    (_, q0), tq0 = timed(lambda: ctx.bf_diag_estimate(sys_, probes, 0, tol, precision=precision))
    (_, ql), tql = timed(lambda: ctx.bf_diag_estimate(sys_, probes, 0, tol, precision=precision, logvar=lv))
    lv_ref = ctx.bf_warm_start_targets(sys_, mu_ref, s_ref)[:, 1].cpu().numpy()
    out["variance"] = {
        "iters_zero": q0["iters"], "iters_learned": ql["iters"], "ms_zero": tq0, "ms_learned": tql,
        "logvar_rmse_learned": float(np.sqrt(np.mean((lv.cpu().numpy() - lv_ref) ** 2))),
        "logvar_rmse_jacobi": float(np.sqrt(np.mean(lv_ref ** 2)))}
    sys_.free()
    band.free()
    return out


def main():
    from synth import make_workload
    ap = argparse.ArgumentParser(description="train the learned warm start on the GPU")
    ap.add_argument("--lam", type=float, default=10.0)
    ap.add_argument("--spheres", type=int, default=100)
    ap.add_argument("--unions", type=int, default=70)
    ap.add_argument("--unions256", type=int, default=30)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", required=True)
    ap.add_argument("--report", default=None)
    ap.add_argument("--checkpoint", default=None, help="training state file, saved every 500 steps")
    ap.add_argument("--resume", action="store_true", help="continue from --checkpoint")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    ctx = Context(dev)
    feats, tgts = [], []
    t0 = time.time()
    scenes = training_scenes(args.spheres, args.unions, args.unions256)
    for k, item in enumerate(scenes):
        name, seed = (item, 0) if isinstance(item, str) else item
        wl = make_workload(name, device=dev, seed=seed)
        f, t = scene_pairs(ctx, wl, args.lam, seed=k)
        feats.append(f)
        tgts.append(t)
        if k % 10 == 0 or name == "union256":
            print(f"[data] scene {k} {name} N={f.shape[0]} ({time.time() - t0:.0f}s)", file=sys.stderr, flush=True)
    feats = torch.cat(feats).contiguous()
    tgts = np.concatenate(tgts)
    print(f"[data] {feats.shape[0]} voxels from {len(scenes)} scenes",
          file=sys.stderr, flush=True)
    params, hist = train(ctx, feats, tgts, steps=args.steps, batch=args.batch, lr=args.lr,
                         checkpoint=args.checkpoint, resume=args.resume)
    np.save(args.out, params)
    report = {"lam": args.lam, "train_voxels": int(feats.shape[0]), "loss_history": hist, "held_out": []}
    for name, seed in (("sphere64", 1000), ("sphere64", 1001), ("union256", 1002)):
        wl = make_workload(name, device=dev, seed=seed)
        for prec in (L.BF_PREC_FP64, L.BF_PREC_MIXED):
            r = evaluate(ctx, wl, args.lam, params, precision=prec)
            r.update(scene=f"{name}/{seed}", precision="fp64" if prec == L.BF_PREC_FP64 else "mixed")
            report["held_out"].append(r)
            print(json.dumps(r), file=sys.stderr, flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()
