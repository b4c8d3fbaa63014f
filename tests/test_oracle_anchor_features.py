"""Pins of the oracle's boundary anchor (eq. 7's lambda_b term and the b0 of
eq. 11) and of every column of the learned start's input features.

The anchor adds lambda_b (x_v - TSDF_v)^2 to the prior energy of each voxel on
the band boundary dB (a band voxel with fewer than 6 band neighbours), so
Q gains lambda_b on those diagonal entries and the right-hand side gains
b0_v = lambda_b TSDF_v.  The tests fix it three ways that do not go through
the oracle's own formulas: the one-voxel and two-voxel posteriors in closed
form, and the quadratic-form identity of the anchored energy on a random band
whose boundary is found by brute force.

The features are pinned on a fixture whose values are derived by hand from
the view depths (``tests/golden/features_wall3.txt``, written with exact
rational arithmetic by ``tests/golden/make_features_wall3.py``).
"""
import itertools
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class _Cam:
    def __init__(self, w, h, fx, fy, cx, cy):
        self.width, self.height, self.fx, self.fy, self.cx, self.cy = w, h, fx, fy, cx, cy


def _sigma(D):
    return 0.0012 + 0.0019 * (D - 0.4) ** 2


def _wall_views(orc, depths):
    """4^3 grid of 0.25 m voxels (low corner -0.5); fronto-parallel walls at the given
    camera depths, seen from (0, 0, -2) along +z, one view per depth."""
    g = orc.grid(4, 0.25, (-0.5,) * 3, 0.5, 0.25)
    cm = orc.cam(_Cam(32, 32, 8.0, 8.0, 15.5, 15.5))
    P = np.zeros((len(depths), 3, 4))
    P[:, :, :3] = np.eye(3)
    P[:, 2, 3] = -2.0
    depth = np.stack([np.full((32, 32), D, dtype=np.float32) for D in depths])
    return g, cm, P, depth


def _keys(orc, cells):
    return np.sort(np.array([orc.morton_encode(*c) for c in cells], dtype=np.uint64))


# ----------------------------------------------------------------- anchor
def test_anchor_single_voxel_closed_form(orc):
    """N = 1 (no band neighbour, so on the boundary): the posterior of one voxel
    with data precision Lambda, data term b, the anchor's pseudo-observation
    TSDF with precision lambda_b and the nugget eps is
    mu = (b + lambda_b t) / (Lambda + lambda_b + eps), s = 1 / (Lambda + lambda_b + eps)."""
    views = [2.1, 2.2, 2.25]
    g, cm, P, depth = _wall_views(orc, views)
    key = _keys(orc, [(1, 2, 2)])  # centre z = 0.125, camera depth 2.125
    Lam, b = orc.assemble(g, cm, depth, P, key)
    nbr, deg = orc.neighbours(4, key)
    assert deg[0] == 0
    Ds = [float(np.float32(D)) for D in views]
    ys = [min(D - 2.125, 0.5) for D in Ds]
    t = sum(ys) / len(ys)            # coarse TSDF: unit-weight mean of the truncated distances
    Lam_ref = sum(1.0 / _sigma(D) ** 2 for D in Ds)
    b_ref = sum(y / _sigma(D) ** 2 for y, D in zip(ys, Ds))
    lam, eps, lam_b = 10.0, 1e-6, 3.0e4
    diag = orc.precision_diag(Lam, deg, lam, eps, lam_b)
    rhs = orc.anchor_rhs(b, deg, np.array([t]), lam_b)
    prec = Lam_ref + lam_b + eps
    assert math.isclose(diag[0], prec, rel_tol=1e-14)
    assert math.isclose(rhs[0], b_ref + lam_b * t, rel_tol=1e-13)
    mu, rep = orc.pcg(nbr, diag, lam, rhs, 1e-15)
    assert math.isclose(mu[0], (b_ref + lam_b * t) / prec, rel_tol=1e-13)
    s = orc.hutchinson(nbr, diag, lam, 1, 0, 1e-15)
    assert math.isclose(s[0], 1.0 / prec, rel_tol=1e-13)
    # without the anchor the posterior ignores the TSDF
    d0 = orc.precision_diag(Lam, deg, lam, eps, 0.0)
    assert math.isclose(d0[0], Lam_ref + eps, rel_tol=1e-14)
    assert orc.anchor_rhs(b, deg, np.array([t]), 0.0)[0] == b[0]


def test_anchor_two_voxels_closed_form(orc):
    """N = 2 with one edge (both voxels on the boundary, degree 1): with
    a_i = Lambda_i + lam + lambda_b + eps and h_i = b_i + lambda_b t_i,
    Q = [[a_1, -lam], [-lam, a_2]], so mu = Q^-1 h and diag(Q^-1) = (a_2, a_1) / det."""
    views = [2.1, 2.2]
    g, cm, P, depth = _wall_views(orc, views)
    keys = _keys(orc, [(1, 2, 2), (1, 2, 3)])  # neighbours along z: camera depths 2.125, 2.375
    Lam, b = orc.assemble(g, cm, depth, P, keys)
    nbr, deg = orc.neighbours(4, keys)
    assert list(deg) == [1, 1]
    Ds = [float(np.float32(D)) for D in views]
    tsdf = np.array([sum(min(D - z, 0.5) for D in Ds) / 2 for z in (2.125, 2.375)])
    lam, eps, lam_b = 2.0e5, 1e-6, 7.0e4
    diag = orc.precision_diag(Lam, deg, lam, eps, lam_b)
    rhs = orc.anchor_rhs(b, deg, tsdf, lam_b)
    a1, a2 = Lam[0] + lam + lam_b + eps, Lam[1] + lam + lam_b + eps
    h1, h2 = b[0] + lam_b * tsdf[0], b[1] + lam_b * tsdf[1]
    det = a1 * a2 - lam * lam
    mu_ref = np.array([(a2 * h1 + lam * h2) / det, (lam * h1 + a1 * h2) / det])
    mu, rep = orc.pcg(nbr, diag, lam, rhs, 1e-15)
    assert np.allclose(mu, mu_ref, rtol=1e-12, atol=0)
    # eq. (12) with N = 2: s_i = S_ii + S_12 m exactly, m the probe average of z_1 z_2
    K = 32
    z = orc.probes(3, K, 2).astype(np.float64)
    m = (z[0] * z[1]).mean()
    S11, S22, S12 = a2 / det, a1 / det, lam / det
    s = orc.hutchinson(nbr, diag, lam, K, 3, 1e-15)
    assert np.allclose(s, [S11 + S12 * m, S22 + S12 * m], rtol=1e-10, atol=0)


def test_anchor_only_on_boundary(orc):
    """A voxel with all 6 band neighbours is interior: the anchor leaves its
    diagonal and right-hand side alone; its 6 neighbours (degree 1) get both."""
    centre = (2, 2, 2)
    cells = [centre] + [tuple(c + d for c, d in zip(centre, off)) for off in
                        ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))]
    keys = _keys(orc, cells)
    nbr, deg = orc.neighbours(5, keys)
    rng = np.random.default_rng(9)
    Lam, b, t = rng.uniform(1, 2, 7), rng.standard_normal(7), rng.standard_normal(7)
    lam, eps, lam_b = 0.5, 1e-6, 4.0
    diag = orc.precision_diag(Lam, deg, lam, eps, lam_b)
    rhs = orc.anchor_rhs(b, deg, t, lam_b)
    for n, k in enumerate(keys):
        interior = orc.morton_decode(int(k)) == centre
        assert deg[n] == (6 if interior else 1)
        want_d = Lam[n] + lam * deg[n] + eps + (0.0 if interior else lam_b)
        want_h = b[n] + (0.0 if interior else lam_b * t[n])
        assert math.isclose(diag[n], want_d, rel_tol=1e-15)
        assert math.isclose(rhs[n], want_h, rel_tol=1e-15, abs_tol=1e-300)


def _brute_boundary(G, cells):
    """Band voxels with fewer than 6 band neighbours, by direct lookup."""
    s = set(cells)
    offs = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))
    return {c for c in cells if sum(tuple(a + d for a, d in zip(c, o)) in s for o in offs) < 6}


def test_anchor_quadratic_form(orc):
    """The anchored prior energy, expanded: for every x,
    x^T Q x - 2 x^T b0 + lambda_b sum_{dB} t^2
      = sum Lambda x^2 + lam sum_edges (x_i - x_j)^2 + lambda_b sum_{dB} (x_i - t_i)^2 + eps sum x^2,
    with Q x from the oracle's operator, b0 = rhs - b, and the boundary and the
    edges found by brute force."""
    G = 7
    rng = np.random.default_rng(12)
    # a solid ball (so interior voxels exist) plus random extra voxels
    cells = [c for c in itertools.product(range(G), repeat=3)
             if sum((x - 3) ** 2 for x in c) <= 5 or rng.random() < 0.25]
    keys = _keys(orc, cells)
    pos = {orc.morton_decode(int(k)): n for n, k in enumerate(keys)}
    nbr, deg = orc.neighbours(G, keys)
    bnd = _brute_boundary(G, list(pos))
    onb = np.zeros(len(keys), dtype=bool)
    for c in bnd:
        onb[pos[c]] = True
    assert 0 < onb.sum() < len(keys)
    edges = [(pos[c], pos[(c[0] + 1, c[1], c[2])]) for c in pos if (c[0] + 1, c[1], c[2]) in pos]
    edges += [(pos[c], pos[(c[0], c[1] + 1, c[2])]) for c in pos if (c[0], c[1] + 1, c[2]) in pos]
    edges += [(pos[c], pos[(c[0], c[1], c[2] + 1)]) for c in pos if (c[0], c[1], c[2] + 1) in pos]
    Lam = rng.uniform(0.5, 2.0, len(keys))
    b = rng.standard_normal(len(keys))
    t = rng.uniform(-0.02, 0.02, len(keys))
    lam, eps, lam_b = 1.5, 1e-6, 2.5
    diag = orc.precision_diag(Lam, deg, lam, eps, lam_b)
    b0 = orc.anchor_rhs(b, deg, t, lam_b) - b
    assert np.all(b0[~onb] == 0.0)
    for _ in range(4):
        x = rng.standard_normal(len(keys))
        lhs = x @ orc.apply_Q(nbr, diag, lam, x) - 2.0 * (x @ b0) + lam_b * (t[onb] ** 2).sum()
        rhs = ((Lam * x * x).sum() + lam * sum((x[i] - x[j]) ** 2 for i, j in edges)
               + lam_b * ((x[onb] - t[onb]) ** 2).sum() + eps * (x * x).sum())
        assert math.isclose(lhs, rhs, rel_tol=1e-11)
    # the anchored energy's minimiser is the solution of Q mu = b + b0: its gradient vanishes
    mu, rep = orc.pcg(nbr, diag, lam, b + b0, 1e-13)
    grad = (2 * Lam * mu + 2 * eps * mu + 2 * lam_b * np.where(onb, mu - t, 0.0) - 2 * b)
    for i, j in edges:
        grad[i] += 2 * lam * (mu[i] - mu[j])
        grad[j] -= 2 * lam * (mu[i] - mu[j])
    assert np.linalg.norm(grad) <= 1e-10 * np.linalg.norm(2 * b)


# ----------------------------------------------------------------- features
def _golden_features():
    rows = {}
    for line in open(os.path.join(GOLDEN, "features_wall3.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows[(int(f[0]), int(f[1]), int(f[2]))] = [float(v) for v in f[3:]]
    return rows


def test_features_multiview_golden(orc):
    """All 12 feature columns of a plus-shaped band (one interior voxel, six arms)
    seen by five fronto-parallel views of walls at 2.1, 2.2, 2.25, 1.6 and 2.45 m
    (the 1.6 m wall occludes the two far layers, the 2.45 m one is truncated at tau
    for the near layer, so W, the sigma statistics and Lambda differ by layer): TSDF/h,
    log(1+W), deg/6, n_obs/T, mean y/h, var y/h^2, mean sigma/h, min sigma/h,
    log(1 + Lambda h^2) and the TSDF central differences, against values derived
    by hand from the view depths."""
    views = [2.1, 2.2, 2.25, 1.6, 2.45]
    g, cm, P, depth = _wall_views(orc, views)
    centre = (1, 2, 2)
    cells = [centre] + [tuple(c + d for c, d in zip(centre, off)) for off in
                        ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))]
    keys = _keys(orc, cells)
    nbr, deg = orc.neighbours(4, keys)
    ijk = np.array([orc.morton_decode(int(k)) for k in keys], dtype=np.int32)
    tsdf, w = orc.tsdf_points(g, cm, depth, P, ijk)
    Lam, b, acc = orc.assemble(g, cm, depth, P, keys, with_acc=True)
    f = orc.features(len(views), 0.25, tsdf, w, nbr, deg, Lam, acc)
    gold = _golden_features()
    assert len(gold) == len(keys)
    for n, c in enumerate(map(tuple, ijk)):
        want = gold[c]
        for col in range(12):
            assert math.isclose(f[n, col], want[col], rel_tol=2e-14, abs_tol=1e-15), (c, col, f[n, col], want[col])
