"""FP64 oracle of the learned warm start's per-voxel MLP (test infrastructure).

The paper names learned priors for geometry regularisation as future work
(Sec. 6 and Sec. 7); the network here is this build's reading of that hook:
12 input features -> 64 -> 64 -> 64 -> 2 outputs, SiLU after each hidden
layer, a fixed input standardisation and a fixed output scaling.  It is
written out plainly in numpy:

* ``forward``/``backward`` in pure FP64 (pinned against finite differences);
* the same with BF16 emulation (round-to-nearest-even of the weights, the
  layer inputs and the back-propagated pre-activation gradients, exactly where
  the GPU kernels feed the matrix cores), for tight checks of those kernels;
* ``adam_step``: Adam (Kingma & Ba, ICLR 2015) with bias correction.

Parameter vector (float32 on the device, float64 here), in this order:
W1[64][12] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[2][64] b4[2]
then the fixed part: in_mean[12] in_std[12] out_mean[2] out_std[2].
Loss: L = 1/(2M) sum_m sum_c (o_mc - t_mc)^2 over a batch of M voxels, with o
in standardised output units.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 12, 64, 2
SHAPES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH, NH)),
          ("b3", (NH,)), ("W4", (NOUT, NH)), ("b4", (NOUT,))]
FIXED = [("in_mean", (NIN,)), ("in_std", (NIN,)), ("out_mean", (NOUT,)), ("out_std", (NOUT,))]
N_TRAIN = sum(int(np.prod(s)) for _, s in SHAPES)            # 9282
N_PARAMS = N_TRAIN + sum(int(np.prod(s)) for _, s in FIXED)  # 9310


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES + FIXED:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(parts[n], dtype=np.float64).ravel() for n, _ in SHAPES + FIXED])


def init(seed: int = 0) -> np.ndarray:
    """He-uniform hidden weights, zero biases, identity standardisation."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[1])
            p[name] = rng.uniform(-lim, lim, size=shp)
        else:
            p[name] = np.zeros(shp)
    p["W4"] *= 0.1
    p["in_mean"], p["in_std"] = np.zeros(NIN), np.ones(NIN)
    p["out_mean"], p["out_std"] = np.zeros(NOUT), np.ones(NOUT)
    return pack(p)


def bf16(x):
    """Round float64 values to the nearest bfloat16 (ties to even), as float64."""
    x = np.asarray(x, dtype=np.float64)
    f = x.astype(np.float32)  # float32 first, as the device rounds float32 values
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X, emulate_bf16=False):
    """Standardised outputs [M][2] and the cache for backward."""
    p = unpack(theta)
    rnd = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    x = (np.asarray(X, dtype=np.float64) - p["in_mean"]) / p["in_std"]
    a = rnd(x)
    cache = {"a0": a}
    for l in (1, 2, 3):
        z = a @ rnd(p[f"W{l}"]).T + p[f"b{l}"]
        cache[f"z{l}"] = z
        a = rnd(silu(z))
        cache[f"a{l}"] = a
    o = a @ rnd(p["W4"]).T + p["b4"]
    return o, cache


def predict(theta, X, emulate_bf16=False):
    """Physical outputs: standardised outputs times out_std plus out_mean."""
    p = unpack(theta)
    o, _ = forward(theta, X, emulate_bf16)
    return o * p["out_std"] + p["out_mean"]


def loss_and_grad(theta, X, Tgt, emulate_bf16=False):
    """Loss and gradient with respect to the trainable parameters (fixed part 0).

    Tgt holds physical targets; they are standardised with out_mean/out_std."""
    p = unpack(theta)
    rnd = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    o, c = forward(theta, X, emulate_bf16)
    M = o.shape[0]
    diff = o - (np.asarray(Tgt, dtype=np.float64) - p["out_mean"]) / p["out_std"]
    L = 0.5 * float((diff * diff).sum()) / M
    g = {n: np.zeros(s) for n, s in SHAPES + FIXED}
    dz = diff / M                                   # dL/do
    g["b4"] = dz.sum(0)
    g["W4"] = rnd(dz).T @ c["a3"]
    da = rnd(dz) @ rnd(p["W4"])
    for l in (3, 2, 1):
        dz = da * dsilu(c[f"z{l}"])
        g[f"b{l}"] = dz.sum(0)
        g[f"W{l}"] = rnd(dz).T @ c[f"a{l - 1}"]
        if l > 1:
            da = rnd(dz) @ rnd(p[f"W{l}"])
    return L, pack(g)


def adam_step(theta, m, v, grad, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of the trainable part; returns new (theta, m, v)."""
    theta, m, v = theta.copy(), m.copy(), v.copy()
    t = slice(0, N_TRAIN)
    m[t] = b1 * m[t] + (1.0 - b1) * grad[t]
    v[t] = b2 * v[t] + (1.0 - b2) * grad[t] * grad[t]
    mh = m[t] / (1.0 - b1 ** step)
    vh = v[t] / (1.0 - b2 ** step)
    theta[t] = theta[t] - lr * mh / (np.sqrt(vh) + eps)
    return theta, m, v
