"""Parity at the benchmark's full size: the 256^3 union scene (40 views at
640x480), run through the library in the configuration bench.py times.

Band keys, TSDF, weights, neighbours, Lambda, b and diag(Q) are compared bit
for bit over the whole band; the FP64 mean and 32-probe variance in relative
L2 (<= 1e-6); the NBV utilities of all 512 candidates and their argmax bit
for bit with shared (mu, s) inputs, and the walk's voxel-visit count.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from tests import gpu_common as gc  # noqa: E402


@pytest.fixture(scope="module")
def full():
    import oracle as O
    import paper_2602_19697_amd as bf
    from synth import make_workload
    wl = make_workload("union256", device=gc.DEV)
    print(f"[union256] rendered {wl.depth.shape}", flush=True)
    ref = O.full_pipeline(wl)
    print(f"[union256] oracle band N={len(ref['keys'])}", flush=True)
    ctx = bf.Context(gc.DEV)
    band, sys_, depth, poses = gc.gpu_system(ctx, wl)
    yield wl, ref, ctx, band, sys_
    sys_.free()
    band.free()
    ctx.close()


def test_fullsize_band_and_assembly_bitexact(full):
    wl, ref, ctx, band, sys_ = full
    a = band.arrays()
    s = sys_.arrays()
    assert band.n == len(ref["keys"]) > 100000
    for name in ("keys", "tsdf", "w", "nbr", "deg"):
        assert np.array_equal(a[name].cpu().numpy(), ref[name]), name
    for name in ("Lambda", "b", "rhs", "diag"):
        assert np.array_equal(s[name].cpu().numpy(), ref[name]), name


def test_fullsize_mean_and_variance(full):
    import oracle as O
    import paper_2602_19697_amd as bf
    wl, ref, ctx, band, sys_ = full
    tol, K = 1e-6, 32
    mu, rep = ctx.bf_pcg_solve(sys_, tol, precision=bf.L.BF_PREC_FP64)
    mu_ref, rep_ref = O.pcg(ref["nbr"], ref["diag"], wl.lam, ref["rhs"], tol)
    err_mu = gc.rel_l2(mu.cpu().numpy(), mu_ref)
    s, prep = ctx.bf_diag_estimate(sys_, K, 0, tol, precision=bf.L.BF_PREC_FP64)
    s_ref = O.hutchinson(ref["nbr"], ref["diag"], wl.lam, K, 0, tol)
    err_s = gc.rel_l2(s.cpu().numpy(), s_ref)
    mum, repm = ctx.bf_pcg_solve(sys_, tol, precision=bf.L.BF_PREC_MIXED)
    sm, prepm = ctx.bf_diag_estimate(sys_, K, 0, tol, precision=bf.L.BF_PREC_MIXED)
    err_mum = gc.rel_l2(mum.cpu().numpy(), mu_ref)
    err_sm = gc.rel_l2(sm.cpu().numpy(), s_ref)
    print(f"[union256] mu err fp64={err_mu:.2e} mixed={err_mum:.2e}; s err fp64={err_s:.2e} mixed={err_sm:.2e}; "
          f"iters {rep['iters']}/{rep_ref['iters']} probes {prep['iters']}")
    assert err_mu <= 1e-6 and err_s <= 1e-6
    assert err_mum <= 1e-4 and err_sm <= 1e-4


def test_fullsize_nbv_all_candidates_bitexact(full):
    """All 512 candidate utilities (eq. 13) and the argmax, bit for bit, with
    shared (mu, s); then the visit count of every ray of every candidate."""
    import oracle as O
    wl, ref, ctx, band, sys_ = full
    mu, _ = O.pcg(ref["nbr"], ref["diag"], wl.lam, ref["rhs"], 1e-6)
    s = O.hutchinson(ref["nbr"], ref["diag"], wl.lam, 4, 0, 1e-6)
    cands = wl.candidates()
    mu_d, s_d = torch.from_numpy(mu).to(gc.DEV), torch.from_numpy(s).to(gc.DEV)
    scores, best = ctx.bf_nbv_score(band, mu_d, s_d, torch.from_numpy(np.ascontiguousarray(cands)).to(gc.DEV),
                                    wl.ray_cam)
    got = scores.cpu().numpy()
    steps_gpu = ctx.bf_nbv_walk_steps()
    q = O.quantize_variance(s)
    want, steps = O.nbv_scores_steps(ref["grid"], O.cam(wl.ray_cam), ref["keys"], mu, q, cands)
    print(f"[union256] NBV best={best} (oracle {O.nbv_argmax(want)}) max={got.max()} "
          f"walk steps {steps_gpu} (oracle {int(steps.sum())})", flush=True)
    assert len(got) == 512 and np.array_equal(got, want)
    assert best == O.nbv_argmax(want)
    assert steps_gpu == int(steps.sum())
