"""GPU parity of the learned warm start: features, the MFMA forward pass, the
backward pass and Adam against the oracle (BF16-emulating FP64 and pure FP64).

Tolerances: the device rounds pre-activations computed in FP32 to BF16 where
the emulating oracle rounds FP64 values, so an activation occasionally lands
one BF16 step (2^-8 relative) apart; such flips are rare and average out over
a layer, so 1e-3 relative L2 bounds the difference from the emulation.
Against pure FP64 the BF16 rounding itself (2^-9 relative per operand,
compounded over four layers) is the error, hence 3e-2.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from tests import gpu_common as gc  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    import paper_2602_19697_amd as bf
    c = bf.Context(gc.DEV)
    yield c
    c.close()


def _params(seed, feat=None):
    from oracle import mlp
    rng = np.random.default_rng(seed)
    th = mlp.init(seed)
    p = mlp.unpack(th)
    for n in ("b1", "b2", "b3", "b4"):
        p[n] = rng.normal(0, 0.1, size=p[n].shape)
    p["W4"] = rng.normal(0, 0.3, size=p["W4"].shape)
    if feat is not None:
        p["in_mean"] = feat.mean(0)
        p["in_std"] = feat.std(0) + 1e-3
    p["out_mean"] = np.array([0.3, -1.0])
    p["out_std"] = np.array([2.0, 0.5])
    return mlp.pack(p).astype(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def sphere_features(ctx):
    import oracle as O
    wl = gc.workload("sphere64")
    ref = gc.oracle_ref("sphere64")
    band, sys_, _, _ = gc.gpu_system(ctx, wl)
    f = ctx.bf_features(sys_)
    f_ref = O.features(wl.T, wl.h, ref["tsdf"], ref["w"], ref["nbr"], ref["deg"], ref["Lambda"], ref["acc"])
    yield wl, ref, band, sys_, f, f_ref
    sys_.free()
    band.free()


def test_features_match_oracle(sphere_features):
    wl, ref, band, sys_, f, f_ref = sphere_features
    got = f.cpu().numpy().astype(np.float64)
    assert got.shape == f_ref.shape
    assert np.allclose(got, f_ref, rtol=2e-7, atol=1e-6)


def test_forward_matches_oracle(ctx, sphere_features):
    from oracle import mlp
    wl, ref, band, sys_, f, f_ref = sphere_features
    th = _params(0, f_ref)
    feat = f.cpu().numpy().astype(np.float64)
    out = ctx.bf_mlp_forward(torch.from_numpy(th.astype(np.float32)).to(gc.DEV), f).cpu().numpy()
    emu = mlp.predict(th, feat, emulate_bf16=True)
    pure = mlp.predict(th, feat)
    e1, e2 = gc.rel_l2(out, emu), gc.rel_l2(out, pure)
    print(f"forward rel err vs emulated {e1:.2e}, vs FP64 {e2:.2e}")
    assert e1 <= 1e-3 and e2 <= 3e-2
    # per-column (two outputs) as well, and a ragged count (not a multiple of 16)
    for c in range(2):
        assert gc.rel_l2(out[:, c], emu[:, c]) <= 1e-3
    n = 1000 + 7
    out2 = ctx.bf_mlp_forward(torch.from_numpy(th.astype(np.float32)).to(gc.DEV), f[:n].contiguous()).cpu().numpy()
    assert np.array_equal(out2, out[:n])


def test_warm_start_outputs(ctx, sphere_features):
    wl, ref, band, sys_, f, f_ref = sphere_features
    th = torch.from_numpy(_params(1, f_ref).astype(np.float32)).to(gc.DEV)
    out = ctx.bf_mlp_forward(th, f).cpu().numpy().astype(np.float64)
    x0, lv = ctx.bf_warm_start(sys_, th, f)
    s = sys_.arrays()
    want = s["rhs"].cpu().numpy() / s["diag"].cpu().numpy() + wl.h * out[:, 0]
    assert np.allclose(x0.cpu().numpy(), want, rtol=1e-12, atol=1e-15)
    assert np.array_equal(lv.cpu().numpy(), out[:, 1].astype(np.float32))
    # features computed in the network's pass: the same bits as through the [N][12] array
    x0f, lvf = ctx.bf_warm_start(sys_, th, None)
    assert torch.equal(x0f, x0) and torch.equal(lvf, lv)


@pytest.mark.parametrize("M", [4096, 1000 + 13])
def test_gradient_matches_oracle(ctx, sphere_features, M):
    from oracle import mlp
    wl, ref, band, sys_, f, f_ref = sphere_features
    th = _params(2, f_ref)
    rng = np.random.default_rng(3)
    N = f.shape[0]
    idx = rng.choice(N, size=M, replace=False).astype(np.int32)
    tgt = rng.normal(size=(N, 2)) * np.array([1.5, 0.4]) + np.array([0.2, -1.1])
    grad, loss = ctx.bf_mlp_grad(torch.from_numpy(th.astype(np.float32)).to(gc.DEV), f,
                                 torch.from_numpy(tgt.astype(np.float32)).to(gc.DEV),
                                 torch.from_numpy(idx).to(gc.DEV))
    feat = f.cpu().numpy().astype(np.float64)[idx]
    T = tgt.astype(np.float32).astype(np.float64)[idx]
    L_emu, g_emu = mlp.loss_and_grad(th, feat, T, emulate_bf16=True)
    L_pure, g_pure = mlp.loss_and_grad(th, feat, T)
    g = grad.cpu().numpy().astype(np.float64)
    e1 = gc.rel_l2(g, g_emu[:mlp.N_TRAIN])
    e2 = gc.rel_l2(g, g_pure[:mlp.N_TRAIN])
    print(f"[M={M}] grad rel err vs emulated {e1:.2e}, vs FP64 {e2:.2e}; loss {loss.item():.6e} vs {L_emu:.6e}")
    assert e1 <= 1e-3 and e2 <= 3e-2
    assert abs(loss.item() - L_emu) <= 1e-4 * L_emu
    # per-block check: each weight matrix and bias on its own
    o = 0
    for name, shp in mlp.SHAPES:
        n = int(np.prod(shp))
        assert gc.rel_l2(g[o:o + n], g_emu[o:o + n]) <= 1e-3, name
        o += n


def test_adam_matches_oracle(ctx):
    from oracle import mlp
    rng = np.random.default_rng(7)
    th = rng.normal(size=mlp.N_PARAMS).astype(np.float32)
    m = (rng.normal(size=mlp.N_PARAMS) * 1e-3).astype(np.float32)
    v = (rng.uniform(size=mlp.N_PARAMS) * 1e-6).astype(np.float32)
    g = (rng.normal(size=mlp.N_PARAMS) * 1e-3).astype(np.float32)
    tt, tm, tv, tg = (torch.from_numpy(a.copy()).to(gc.DEV) for a in (th, m, v, g))
    ctx.bf_adam_step(tt, tm, tv, tg[:mlp.N_TRAIN].contiguous(), 5, lr=1e-3)
    th2, m2, v2 = mlp.adam_step(th.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                                g.astype(np.float64), 5, lr=1e-3)
    assert np.allclose(tt.cpu().numpy(), th2, rtol=1e-6, atol=1e-7)
    assert np.allclose(tm.cpu().numpy(), m2, rtol=1e-5, atol=1e-10)
    assert np.array_equal(tt.cpu().numpy()[mlp.N_TRAIN:], th[mlp.N_TRAIN:])


def test_training_resumes_bit_for_bit(tmp_path):
    """A run interrupted after 10 of 20 Adam steps and resumed from its
    checkpoint ends with the same parameters as an uninterrupted run."""
    import paper_2602_19697_amd as bf
    from paper_2602_19697_amd import learned
    ctx = bf.Context(gc.DEV)
    wl = gc.workload("sphere64")
    feat, tgt = learned.scene_pairs(ctx, wl, 1e5, probes=4)
    ck = str(tmp_path / "ck.npz")
    full, hist_full = learned.train(ctx, feat, tgt, steps=20, batch=2048, log_every=5)
    part, _ = learned.train(ctx, feat, tgt, steps=20, batch=2048, log_every=5, checkpoint=ck, checkpoint_every=10,
                            stop_at=10)
    assert not np.array_equal(part, full)
    resumed, hist_res = learned.train(ctx, feat, tgt, steps=20, batch=2048, log_every=5, checkpoint=ck,
                                      checkpoint_every=10, resume=True)
    assert np.array_equal(resumed, full)
    assert hist_res == hist_full
    ctx.close()
