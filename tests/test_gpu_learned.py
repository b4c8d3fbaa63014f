"""What the trained warm-start network gains over the method without it.

The committed networks (paper_2602_19697_amd/weights/) were trained on the GPU
by the library's own forward, backward and Adam kernels on solves of 200
seeded training scenes (learned.py).  Here they run on held-out scenes (seeds
the training never saw).  The solver stays the judge: from any start PCG runs
to the same tolerance, so the answers must match the oracle as without the
network; the network may only move the start closer and cut iterations.

Training report at lambda = 1e5 (warm_start_lam1e5.json), held-out scenes:
sphere64: start error 0.26 (Jacobi start rhs/diag) -> 0.04 (learned), mean
iterations to 1e-6 8 -> 7, log-variance error 0.030 -> 0.020, probe
iterations 9 -> 8; union256: start error 0.22 -> 0.035, mean iterations
13 -> 11, log-variance error 0.035 -> 0.018, probe iterations 17 -> 16.
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


def _setup(ctx, lam, seed=1000):
    import oracle as O
    from paper_2602_19697_amd import learned
    wl = gc.workload("sphere64", seed)
    ref = gc.oracle_ref("sphere64", seed)
    band, sys_, _, _ = gc.gpu_system(ctx, wl, lam=lam)
    diag = O.precision_diag(ref["Lambda"], ref["deg"], lam, wl.eps)
    mu_ref, _ = O.pcg(ref["nbr"], diag, lam, ref["rhs"], 1e-12)
    feat = ctx.bf_features(sys_)
    learned_p = torch.from_numpy(np.load(learned.weights_path(lam))).to(gc.DEV)
    zero_p = torch.from_numpy(learned.zero_params()).to(gc.DEV)
    return wl, ref, band, sys_, diag, mu_ref, feat, learned_p, zero_p


@pytest.mark.parametrize("lam", [10.0, 1e5])
def test_learned_mean_start(ctx, lam):
    wl, ref, band, sys_, diag, mu_ref, feat, learned_p, zero_p = _setup(ctx, lam)
    x_jac, _ = ctx.bf_warm_start(sys_, zero_p, feat, logvar=False)
    x_nn, _ = ctx.bf_warm_start(sys_, learned_p, feat, logvar=False)
    # the zero network is exactly the Jacobi start rhs / diag
    s = sys_.arrays()
    assert torch.equal(x_jac, s["rhs"] / s["diag"])
    e_jac = gc.rel_l2(x_jac.cpu().numpy(), mu_ref)
    e_nn = gc.rel_l2(x_nn.cpu().numpy(), mu_ref)
    results = {}
    for name, x0 in (("zero", None), ("jacobi", x_jac), ("learned", x_nn)):
        mu, rep = ctx.bf_pcg_solve(sys_, 1e-8, precision=0, x0=x0)
        results[name] = rep["iters"]
        assert rep["status"] == 0 and gc.rel_l2(mu.cpu().numpy(), mu_ref) <= 1e-6
    print(f"[lambda={lam:g}] start error jacobi {e_jac:.2e} learned {e_nn:.2e}; iterations {results}")
    assert e_nn < 0.5 * e_jac
    assert results["learned"] <= results["jacobi"] <= results["zero"]
    if lam >= 1e5:
        assert results["learned"] < results["zero"]
    sys_.free()
    band.free()


def test_learned_logvar_start(ctx):
    import oracle as O
    lam = 1e5
    wl, ref, band, sys_, diag, mu_ref, feat, learned_p, zero_p = _setup(ctx, lam)
    s64 = O.hutchinson(ref["nbr"], diag, lam, 64, 4242, 1e-10)
    lv_ref = np.log(np.clip(s64 * diag, 1e-3, 1e3))
    _, lv = ctx.bf_warm_start(sys_, learned_p, feat, mean=False)
    rmse_nn = float(np.sqrt(np.mean((lv.cpu().numpy() - lv_ref) ** 2)))
    rmse_jac = float(np.sqrt(np.mean(lv_ref ** 2)))  # the start u0 = z / diag has log-variance 0
    s0, rep0 = ctx.bf_diag_estimate(sys_, 16, 7, 1e-8)
    s1, rep1 = ctx.bf_diag_estimate(sys_, 16, 7, 1e-8, logvar=lv)
    s_ref = O.hutchinson(ref["nbr"], diag, lam, 16, 7, 1e-12)
    print(f"log-variance rmse jacobi {rmse_jac:.4f} learned {rmse_nn:.4f}; probe iterations "
          f"{rep0['iters']} -> {rep1['iters']}")
    assert rmse_nn < rmse_jac
    assert rep1["used_warm_start"] == 1 and rep1["iters"] <= rep0["iters"]
    assert gc.rel_l2(s1.cpu().numpy(), s_ref) <= 1e-6 and gc.rel_l2(s0.cpu().numpy(), s_ref) <= 1e-6
    sys_.free()
    band.free()
