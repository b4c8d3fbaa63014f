"""Pins of the MLP oracle: finite differences, an independent bfloat16
conversion, Adam's first step in closed form."""
import numpy as np
import pytest

from oracle import mlp


def _theta(seed=0):
    rng = np.random.default_rng(seed)
    th = mlp.init(seed)
    p = mlp.unpack(th)
    for n in ("b1", "b2", "b3", "b4"):
        p[n] = rng.normal(0, 0.1, size=p[n].shape)
    p["in_mean"] = rng.normal(0, 1, size=12)
    p["in_std"] = rng.uniform(0.5, 2.0, size=12)
    p["out_mean"] = rng.normal(0, 1, size=2)
    p["out_std"] = rng.uniform(0.5, 2.0, size=2)
    return mlp.pack(p)


def test_sizes():
    assert mlp.N_TRAIN == 9282 and mlp.N_PARAMS == 9310


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    th = _theta(1)
    X = rng.normal(size=(7, 12))
    T = rng.normal(size=(7, 2))
    L, g = mlp.loss_and_grad(th, X, T)
    idx = np.concatenate([rng.choice(mlp.N_TRAIN, 300, replace=False), [9280, 9281, 0, 767, 768]])
    h = 1e-6
    fd = np.empty(len(idx))
    for n, i in enumerate(idx):
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd[n] = (mlp.loss_and_grad(tp, X, T)[0] - mlp.loss_and_grad(tm, X, T)[0]) / (2 * h)
    assert np.linalg.norm(fd - g[idx]) / np.linalg.norm(g[idx]) < 1e-6
    assert np.all(g[mlp.N_TRAIN:] == 0)


def test_loss_closed_form_constant_network():
    """With zero last-layer weights the output is b4 for every voxel."""
    th = _theta(2)
    p = mlp.unpack(th)
    p["W4"][:] = 0.0
    th = mlp.pack(p)
    X = np.random.default_rng(3).normal(size=(5, 12))
    T = np.random.default_rng(4).normal(size=(5, 2))
    Tn = (T - p["out_mean"]) / p["out_std"]
    L, g = mlp.loss_and_grad(th, X, T)
    assert np.isclose(L, 0.5 * ((p["b4"] - Tn) ** 2).sum() / 5, rtol=1e-14)
    assert np.allclose(mlp.unpack(g)["b4"], (p["b4"] - Tn).mean(0), rtol=1e-14)
    assert np.allclose(mlp.predict(th, X), p["b4"] * p["out_std"] + p["out_mean"], rtol=1e-14)


def test_bf16_rounding_against_torch_and_ties():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-20, 20, size=5000),
                        [1.0, -2.5, 0.0, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x.astype(np.float64)), ref)
    # ties go to the even mantissa
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(6)
    th = rng.normal(size=mlp.N_PARAMS)
    g = rng.normal(size=mlp.N_PARAMS)
    m = np.zeros(mlp.N_PARAMS)
    v = np.zeros(mlp.N_PARAMS)
    th2, m2, v2 = mlp.adam_step(th, m, v, g, 1, lr=1e-2, eps=1e-8)
    t = slice(0, mlp.N_TRAIN)
    assert np.allclose(th2[t], th[t] - 1e-2 * g[t] / (np.abs(g[t]) + 1e-8), rtol=1e-12)
    assert np.array_equal(th2[mlp.N_TRAIN:], th[mlp.N_TRAIN:])


def test_dsilu_matches_finite_differences():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.allclose(mlp.dsilu(z), fd, rtol=1e-7, atol=1e-9)
