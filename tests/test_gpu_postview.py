"""Post-view NBV utility (Sec. 3.8, eq. 13) on the GPU against the oracle.

* bf_predict_depth: the predicted depth maps bit for bit, on the oracle's mu.
* bf_assemble_more: appending views equals assembling all views at once, bit
  for bit (Lambda, b, rhs, diag(Q), statistics), and the oracle's Lambda +
  the predicted view's Lambda.
* bf_nbv_postview: s' and U against the oracle's FP64 post-view solves with
  the same probes, FP64 and mixed precision; the selection among candidates.
"""
import math

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


def _setup(ctx, name, lam=None):
    import oracle as O
    wl = gc.workload(name)
    ref = gc.oracle_ref(name)
    lam = wl.lam if lam is None else lam
    band, sys_, depth, poses = gc.gpu_system(ctx, wl, lam=lam)
    diag = O.precision_diag(ref["Lambda"], ref["deg"], lam, wl.eps)
    mu, _ = O.pcg(ref["nbr"], diag, lam, O.anchor_rhs(ref["b"], ref["deg"], ref["tsdf"], 0.0), 1e-12)
    return wl, ref, band, sys_, depth, poses, diag, mu


@pytest.mark.parametrize("name", ["tiny", "sphere64", "union128"])
def test_predict_depth_bitexact(ctx, name):
    import oracle as O
    wl, ref, band, sys_, _, _, _, mu = _setup(ctx, name)
    cands = wl.candidates()
    mu_d = torch.from_numpy(mu).to(gc.DEV)
    hits = 0
    for c in (0, 7, 100, 311):
        P = np.ascontiguousarray(cands[c].reshape(3, 4))
        got = ctx.bf_predict_depth(band, mu_d, torch.from_numpy(P).to(gc.DEV), wl.cam).cpu().numpy()
        want = O.pred_depth(ref["grid"], ref["cam"], ref["keys"], mu, P)
        assert np.array_equal(got, want), (name, c)
        hits += int((want > 0).sum())
    print(f"[pred depth {name}] {hits} pixels with a return", flush=True)
    assert hits > 0
    sys_.free()
    band.free()


def test_assemble_more_equals_all_views(ctx):
    import oracle as O
    import paper_2602_19697_amd as bf
    wl, ref, band, sys_, depth, poses, _, mu = _setup(ctx, "sphere64")
    cands = wl.candidates()
    views = [np.ascontiguousarray(cands[c].reshape(3, 4)) for c in (2, 40)]
    pred = [O.pred_depth(ref["grid"], ref["cam"], ref["keys"], mu, P) for P in views]
    nd = torch.from_numpy(np.stack(pred)).to(gc.DEV)
    npose = torch.from_numpy(np.stack(views)).to(gc.DEV)
    noise = bf.noise_struct(*wl.noise)
    more = ctx.bf_assemble_more(sys_, wl.cam, nd, npose, noise)
    allv = ctx.bf_assemble(band, wl.cam, torch.cat([depth, nd]), torch.cat([poses, npose]), noise, wl.lam, wl.eps)
    a, b = more.arrays(), allv.arrays()
    for k in ("Lambda", "b", "rhs", "diag", "diag32", "acc"):
        assert torch.equal(a[k], b[k]), k
    dl = sum(O.assemble(ref["grid"], ref["cam"], pred[i][None], views[i][None], ref["keys"], noise=wl.noise)[0]
             for i in range(1))
    one = ctx.bf_assemble_more(sys_, wl.cam, nd[:1], npose[:1], noise)
    assert np.array_equal(one.arrays()["Lambda"].cpu().numpy(), ref["Lambda"] + dl)
    # appending nothing reproduces the system
    same = ctx.bf_assemble_more(sys_, wl.cam, nd[:0], npose[:0], noise)
    for k in ("Lambda", "rhs", "diag", "acc"):
        assert torch.equal(same.arrays()[k], sys_.arrays()[k]), k
    for s in (more, allv, one, same, sys_):
        s.free()
    band.free()


@pytest.mark.parametrize("prec,tol,bound", [(0, 1e-10, 1e-6), (1, 1e-6, 1e-4)])
def test_postview_matches_oracle(ctx, prec, tol, bound):
    import oracle as O
    import paper_2602_19697_amd as bf
    lam, K, seed = 1e5, 16, 5
    precision = bf.L.BF_PREC_FP64 if prec == 0 else bf.L.BF_PREC_MIXED
    wl, ref, band, sys_, _, _, diag, mu = _setup(ctx, "sphere64", lam=lam)
    s = O.hutchinson(ref["nbr"], diag, lam, K, seed, 1e-12)
    cands = wl.candidates()
    which = [3, 17, 64, 200]
    eps_band = 0.02
    U, best, s_post, reps = ctx.bf_nbv_postview(sys_, torch.from_numpy(mu).to(gc.DEV), torch.from_numpy(s).to(gc.DEV),
                                                torch.from_numpy(np.ascontiguousarray(cands)).to(gc.DEV), which,
                                                wl.cam, bf.noise_struct(*wl.noise), K, seed, tol, precision=precision,
                                                eps_band=eps_band, warm=(prec == 1), keep_s=True)
    scale = math.fsum(np.abs(s)[np.abs(mu) <= eps_band])
    Uo = []
    for i, c in enumerate(which):
        u, sp, _, _, _ = O.nbv_postview(ref["grid"], ref["cam"], ref["keys"], ref["nbr"], ref["deg"], ref["Lambda"],
                                        lam, wl.eps, mu, s, cands[c].reshape(3, 4), K, seed, 1e-12,
                                        eps_band=eps_band, noise=wl.noise)
        Uo.append(u)
        err = gc.rel_l2(s_post[i].cpu().numpy(), sp)
        print(f"[postview prec={prec}] cand {c}: U {U[i]:.6e} (oracle {u:.6e}) s' err {err:.2e} "
              f"iters {reps[i]['iters']} warm {reps[i]['used_warm_start']}", flush=True)
        assert reps[i]["status"] == 0 and err <= bound
        assert abs(U[i] - u) <= bound * scale
    # the selection: the oracle's argmax whenever its margin exceeds the tolerance
    order = np.argsort(Uo)[::-1]
    if Uo[order[0]] - Uo[order[1]] > 2 * bound * scale:
        assert best == which[int(order[0])]
    sys_.free()
    band.free()


def test_postview_edge_cases(ctx):
    import paper_2602_19697_amd as bf
    wl, ref, band, sys_, _, _, diag, mu = _setup(ctx, "tiny")
    cands = torch.from_numpy(np.ascontiguousarray(wl.candidates())).to(gc.DEV)
    m = torch.from_numpy(mu).to(gc.DEV)
    s = torch.ones(sys_.n, dtype=torch.float64, device=gc.DEV)
    noise = bf.noise_struct(*wl.noise)
    U, best, _, _ = ctx.bf_nbv_postview(sys_, m, s, cands, [], wl.cam, noise, 4, 0, 1e-8)
    assert U == [] and best == -1
    with pytest.raises(bf.BFError) as e:
        ctx.bf_nbv_postview(sys_, m, s, cands, [int(cands.shape[0])], wl.cam, noise, 4, 0, 1e-8)
    assert e.value.status == bf.L.BF_ERR_INVALID_ARG
    with pytest.raises(bf.BFError) as e:
        ctx.bf_nbv_postview(sys_, m, s, cands, [0], wl.cam, noise, 4, 0, 1e-8, eps_band=-1.0)
    assert e.value.status == bf.L.BF_ERR_INVALID_ARG
    # ties keep the first candidate: the same pose twice
    U, best, _, _ = ctx.bf_nbv_postview(sys_, m, s, cands, [9, 9], wl.cam, noise, 4, 0, 1e-8)
    assert U[0] == U[1] and best == 9
    sys_.free()
    band.free()
