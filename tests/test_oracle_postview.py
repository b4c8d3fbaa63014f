"""Pins of the oracle's post-view utility (Sec. 3.8, eq. 13: U = sum of s - s'
over Omega_eps, s' the variance once the candidate's view is fused).

* The predicted depth of each pixel is the camera-z depth of the first band
  voxel with mu <= 0 on its ray: checked against dense sampling of the ray.
* Fusing the predicted view by adding its Lambda to the system's equals
  assembling all T + 1 views at once (eqs. 3-5, 10-11), bit for bit.
* lambda = 0 makes Q diagonal, where the Hutchinson estimate is exact
  (z_i^2 = 1): U is then sum (1/diag - 1/diag').
* With coupling, U equals the same probes' estimator evaluated with dense
  inverses of Q and Q' (Cholesky), on a small band.
"""
import math

import numpy as np
import scipy.linalg

from tests.test_oracle_pins import _Cam, _full_band, _sample_voxels


def _ball_mu(orc, keys, centre, r2):
    mu = np.ones(len(keys))
    for n, k in enumerate(keys):
        c = orc.morton_decode(int(k))
        if sum((x - y) ** 2 for x, y in zip(c, centre)) < r2:
            mu[n] = -1.0
    return mu


def test_pred_depth_dense_sampling(orc):
    G, h = 8, 0.125
    g = orc.grid(G, h, (-0.5,) * 3, 0.5, 0.25)
    keys = _full_band(orc, G)
    mu = _ball_mu(orc, keys, (3.6, 3.4, 3.5), 5.0)
    pos = {orc.morton_decode(int(k)): n for n, k in enumerate(keys)}
    W, H, f, cx, cy = 7, 5, 5.0, 3.13, 1.87
    cm = orc.cam(_Cam(W, H, f, f, cx, cy))
    # camera at (0.02, -0.03, -1.4) looking along +z, and one looking along -x
    Rx = np.array([[0.0, 0.0, -1.0], [0.0, 1.0, 0.0], [1.0, 0.0, 0.0]])
    poses = [np.hstack([np.eye(3), [[0.02], [-0.03], [-1.4]]]), np.hstack([Rx, [[1.4], [0.01], [0.04]]])]
    hits = 0
    for P in poses:
        depth = orc.pred_depth(g, cm, keys, mu, P)
        assert depth.shape == (H, W) and depth.dtype == np.float32
        Pf = P.reshape(12)
        for row in range(H):
            for col in range(W):
                d = P[:, :3] @ np.array([(col - cx) / f, (row - cy) / f, 1.0])
                want = 0.0
                for c in _sample_voxels(g, P[:, 3], d):
                    if mu[pos[c]] <= 0.0:
                        x = [g.origin[a] + (c[a] + 0.5) * h for a in range(3)]
                        dx, dy, dz = x[0] - Pf[3], x[1] - Pf[7], x[2] - Pf[11]
                        want = float(np.float32((Pf[2] * dx + Pf[6] * dy) + Pf[10] * dz))
                        break
                assert float(depth[row, col]) == want, (row, col)
                hits += want > 0.0
    assert hits >= 6  # the ball is seen from both poses


def _tiny(orc):
    from synth import make_workload
    wl = make_workload("tiny")
    ref = orc.full_pipeline(wl, with_acc=True)
    mu, _ = orc.pcg(ref["nbr"], ref["diag"], wl.lam, ref["rhs"], 1e-12)
    return wl, ref, mu


def test_postview_fusion_equals_assembling_all_views(orc):
    wl, ref, mu = _tiny(orc)
    cands = wl.candidates()
    P = cands[3].reshape(3, 4)
    s = orc.hutchinson(ref["nbr"], ref["diag"], wl.lam, 4, 1, 1e-10)
    U, s_post, dlam, depth, diag_post = orc.nbv_postview(ref["grid"], ref["cam"], ref["keys"], ref["nbr"], ref["deg"],
                                                        ref["Lambda"], wl.lam, wl.eps, mu, s, P, 4, 1, 1e-10,
                                                        noise=wl.noise)
    assert (dlam > 0).sum() > 100 and (depth > 0).sum() > 100
    depth_all = np.concatenate([wl.depth, depth[None]]).astype(np.float32)
    poses_all = np.concatenate([wl.poses, P[None]])
    Lam_all, b_all = orc.assemble(ref["grid"], ref["cam"], depth_all, poses_all, ref["keys"], noise=wl.noise)
    assert np.array_equal(ref["Lambda"] + dlam, Lam_all)
    assert np.array_equal(diag_post, orc.precision_diag(Lam_all, ref["deg"], wl.lam, wl.eps))
    # a view adds observations only: the variance cannot grow anywhere in expectation, and U > 0 here
    assert U > 0.0


def test_postview_closed_form_without_coupling(orc):
    wl, ref, mu = _tiny(orc)
    lam = 0.0
    diag = orc.precision_diag(ref["Lambda"], ref["deg"], lam, wl.eps)
    s = orc.hutchinson(ref["nbr"], diag, lam, 3, 7, 1e-13)
    assert np.allclose(s, 1.0 / diag, rtol=1e-13, atol=0.0)
    P = wl.candidates()[5].reshape(3, 4)
    eps_band = 0.05
    U, s_post, dlam, _, diag_post = orc.nbv_postview(ref["grid"], ref["cam"], ref["keys"], ref["nbr"], ref["deg"],
                                                    ref["Lambda"], lam, wl.eps, mu, s, P, 3, 7, 1e-13,
                                                    eps_band=eps_band, noise=wl.noise)
    sel = np.abs(mu) <= eps_band
    want = math.fsum((1.0 / diag - 1.0 / diag_post)[sel])
    assert want > 0.0 and sel.sum() < len(mu)
    assert abs(U - want) <= 1e-12 * want


def test_postview_dense_inverse_same_probes(orc):
    wl, ref, mu = _tiny(orc)
    N, K, seed = len(ref["keys"]), 6, 3
    s = orc.hutchinson(ref["nbr"], ref["diag"], wl.lam, K, seed, 1e-13)
    P = wl.candidates()[11].reshape(3, 4)
    U, s_post, dlam, _, diag_post = orc.nbv_postview(ref["grid"], ref["cam"], ref["keys"], ref["nbr"], ref["deg"],
                                                    ref["Lambda"], wl.lam, wl.eps, mu, s, P, K, seed, 1e-13,
                                                    noise=wl.noise)

    def dense(diag):
        Q = np.diag(diag)
        for v in range(N):
            for u in ref["nbr"][v]:
                if u >= 0:
                    Q[v, u] = -wl.lam
        return Q

    Z = orc.probes(seed, K, N).astype(np.float64)
    c1 = scipy.linalg.cho_factor(dense(ref["diag"]))
    c2 = scipy.linalg.cho_factor(dense(diag_post))
    s_d = (Z * scipy.linalg.cho_solve(c1, Z)).mean(axis=1)
    s2_d = (Z * scipy.linalg.cho_solve(c2, Z)).mean(axis=1)
    assert np.max(np.abs(s_post - s2_d)) <= 1e-9 * np.max(np.abs(s2_d))
    U_d = math.fsum(s_d - s2_d)
    assert U_d > 0.0
    assert abs(U - U_d) <= 1e-8 * math.fsum(np.abs(s_d))
