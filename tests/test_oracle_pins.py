"""Pins of the FP64 CPU oracle against mathematics, not against itself.

Each test fixes a value the paper's equations determine independently of the
oracle's code: hand-derived fixtures, closed-form posteriors, invariants of Q,
dense factorisations on tiny bands and brute force.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class _Cam:
    def __init__(self, w, h, fx, fy, cx, cy):
        self.width, self.height, self.fx, self.fy, self.cx, self.cy = w, h, fx, fy, cx, cy


def _pose(t, R=None):
    P = np.zeros((3, 4))
    P[:, :3] = np.eye(3) if R is None else R
    P[:, 3] = t
    return P


def _wall(orc, G, h, z_plane, cam_z, tau, band, fx=16.0, W=64, views=1):
    g = orc.grid(G, h, (-G * h / 2,) * 3, tau, band)
    cm = orc.cam(_Cam(W, W, fx, fx, (W - 1) / 2, (W - 1) / 2))
    P = np.stack([_pose((0.0, 0.0, cam_z))] * views)
    D = np.float32(z_plane - cam_z)
    assert float(D) == z_plane - cam_z  # dyadic, exactly representable
    depth = np.full((views, W, W), D, dtype=np.float32)
    return g, cm, P, depth


# ----------------------------------------------------------------- fixtures
def test_wall4_golden(orc):
    """Sec. 3.3 / eq. (1) on the hand-enumerated 4^3 fixture."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "wall4.txt")) if l[0] != "#"]
    g = orc.grid(4, 0.25, (-0.5,) * 3, 0.5, 0.25)
    cm = orc.cam(_Cam(32, 32, 8.0, 8.0, 15.5, 15.5))
    P = _pose((0.0, 0.0, -2.0))[None]
    depth = np.full((1, 32, 32), 2.125, dtype=np.float32)
    td, wd = orc.tsdf_dense(g, cm, depth, P)
    for k, t, w, inb in rows:
        k = int(k)
        assert np.all(td[k] == float(t)) and np.all(wd[k] == int(w))
    keys, bt, bw = orc.band(g, td, wd)
    assert len(keys) == sum(16 * int(r[3]) for r in rows) == 48


def test_splitmix_published_vectors(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) if l[0] != "#"]
    for n, v in rows:
        assert orc.splitmix_output(0, int(n)) == int(v, 16)


# ----------------------------------------------------------------- Morton
def test_morton_roundtrip_and_order(orc):
    rng = np.random.default_rng(1)
    for i, j, k in rng.integers(0, 1 << 20, size=(200, 3)):
        assert orc.morton_decode(orc.morton_encode(i, j, k)) == (i, j, k)
    # brute force: bit interleaving of a 4^3 grid
    for i, j, k in itertools.product(range(4), repeat=3):
        want = sum(((i >> b) & 1) << (3 * b) | ((j >> b) & 1) << (3 * b + 1) |
                   ((k >> b) & 1) << (3 * b + 2) for b in range(2))
        assert orc.morton_encode(i, j, k) == want


# ----------------------------------------------------------------- TSDF / band
@pytest.mark.parametrize("z_index,beta,expect_slabs", [(8, 3, 7), (8, 2, 5)])
def test_planar_wall_band(orc, z_index, beta, expect_slabs):
    """Dyadic fronto-parallel wall, noise-free: the arithmetic is exact, the TSDF is
    the true signed distance and the band is whole slabs, including the inclusive
    boundary tie |TSDF| == beta h."""
    G, h = 16, 2.0 ** -6
    z_plane = -G * h / 2 + (z_index + 0.5) * h
    g, cm, P, depth = _wall(orc, G, h, z_plane, -1.0, 4 * h, beta * h)
    td, wd = orc.tsdf_dense(g, cm, depth, P)
    for k in range(G):
        d = (z_index - k) * h
        if d < -4 * h:
            assert np.all(wd[k] == 0)
        else:
            assert np.all(wd[k] == 1)
            assert np.all(td[k] == min(d, 4 * h))
    keys, bt, bw = orc.band(g, td, wd)
    assert len(keys) == G * G * expect_slabs
    assert np.all(np.diff(keys.astype(np.uint64)) > 0)
    assert np.all(np.abs(bt) <= beta * h)


def test_tsdf_range_and_views(orc):
    """TSDF in [-tau, tau]; two identical views leave the average unchanged."""
    G, h = 16, 2.0 ** -6
    z_plane = -G * h / 2 + 8.5 * h
    g, cm, P, depth = _wall(orc, G, h, z_plane, -1.0, 4 * h, 3 * h, views=2)
    td2, wd2 = orc.tsdf_dense(g, cm, depth, P)
    td1, wd1 = orc.tsdf_dense(g, cm, depth[:1], P[:1])
    assert np.array_equal(td1, td2) and np.array_equal(wd2, 2 * wd1)
    assert np.all(np.abs(td2) <= 4 * h)


def test_invalid_pixels_ignored(orc):
    G, h = 16, 2.0 ** -6
    g, cm, P, depth = _wall(orc, G, h, 0.0078125, -1.0, 4 * h, 3 * h)
    depth[:] = 0.0
    td, wd = orc.tsdf_dense(g, cm, depth, P)
    assert np.all(wd == 0)
    keys, _, _ = orc.band(g, td, wd)
    assert len(keys) == 0


# ----------------------------------------------------------------- neighbours
def _brute_neighbours(G, keys, orc):
    pos = {orc.morton_decode(k): n for n, k in enumerate(keys)}
    nbr = np.full((len(keys), 6), -1, dtype=np.int32)
    offs = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    for (i, j, k), n in pos.items():
        for s, (a, b, c) in enumerate(offs):
            nbr[n, s] = pos.get((i + a, j + b, k + c), -1)
    return nbr


def test_neighbours_bruteforce_and_symmetry(orc):
    rng = np.random.default_rng(3)
    G = 8
    cells = [c for c in itertools.product(range(G), repeat=3) if rng.random() < 0.4]
    keys = np.sort(np.array([orc.morton_encode(*c) for c in cells], dtype=np.uint64))
    nbr, deg = orc.neighbours(G, keys)
    assert np.array_equal(nbr, _brute_neighbours(G, keys, orc))
    assert np.array_equal(deg, (nbr >= 0).sum(1))
    for v in range(len(keys)):
        for a in range(3):
            u = nbr[v, 2 * a]
            if u >= 0:
                assert nbr[u, 2 * a + 1] == v


# ----------------------------------------------------------------- posterior
def _single_voxel_obs(orc, views):
    """One voxel observed by several fronto-parallel views of walls at given depths."""
    G, h = 4, 0.25
    g = orc.grid(G, h, (-0.5,) * 3, 0.5, 0.25)
    cm = orc.cam(_Cam(32, 32, 8.0, 8.0, 15.5, 15.5))
    P = np.stack([_pose((0.0, 0.0, -2.0))] * len(views))
    depth = np.stack([np.full((32, 32), D, dtype=np.float32) for D in views])
    key = np.array([orc.morton_encode(1, 2, 2)], dtype=np.uint64)  # centre z = 0.125
    return g, cm, P, depth, key


def _sigma(D):
    return 0.0012 + 0.0019 * (D - 0.4) ** 2


@pytest.mark.parametrize("views", [[2.125], [2.1, 2.2, 2.25]])
def test_scalar_posterior_closed_form(orc, views):
    """N = 1: prior N(0, 1/eps) and independent Gaussian observations y_t with
    variance sigma(D_t)^2 give the textbook posterior precision sum 1/sigma^2 + eps
    and mean sum(y/sigma^2)/precision (eqs. 9-11)."""
    g, cm, P, depth, key = _single_voxel_obs(orc, views)
    eps, lam = 1e-6, 10.0
    Lam, b = orc.assemble(g, cm, depth, P, key)
    nbr, deg = orc.neighbours(4, key)
    diag = orc.precision_diag(Lam, deg, lam, eps)
    mu, rep = orc.pcg(nbr, diag, lam, b, 1e-14)
    z = 0.125 + 2.0
    ys = [min(float(np.float32(D)) - z, 0.5) for D in views]
    prec = sum(1.0 / _sigma(float(np.float32(D))) ** 2 for D in views) + eps
    mean = sum(y / _sigma(float(np.float32(D))) ** 2 for y, D in zip(ys, views)) / prec
    assert math.isclose(diag[0], prec, rel_tol=1e-14)
    assert math.isclose(mu[0], mean, rel_tol=1e-13)
    s = orc.hutchinson(nbr, diag, lam, 1, 0, 1e-14)
    assert math.isclose(s[0], 1.0 / prec, rel_tol=1e-13)


def test_two_voxel_closed_form(orc):
    """N = 2 with one edge: Q = [[L1+lam+eps, -lam], [-lam, L2+lam+eps]] and the
    posterior mean and variances follow from the explicit 2x2 inverse."""
    g, cm, P, depth, _ = _single_voxel_obs(orc, [2.1, 2.2])
    keys = np.sort(np.array([orc.morton_encode(1, 2, 2), orc.morton_encode(2, 2, 2)],
                            dtype=np.uint64))
    Lam, b = orc.assemble(g, cm, depth, P, keys)
    nbr, deg = orc.neighbours(4, keys)
    assert list(deg) == [1, 1]
    lam, eps = 3.0e5, 1e-6
    diag = orc.precision_diag(Lam, deg, lam, eps)
    a11, a22 = Lam[0] + lam + eps, Lam[1] + lam + eps
    det = a11 * a22 - lam * lam
    mu_ref = np.array([(a22 * b[0] + lam * b[1]) / det, (lam * b[0] + a11 * b[1]) / det])
    mu, rep = orc.pcg(nbr, diag, lam, b, 1e-15)
    assert np.allclose(mu, mu_ref, rtol=1e-12, atol=0)
    # eq. (12) with N = 2: s_1 = S_11 + S_12 m and s_2 = S_22 + S_12 m exactly, where
    # S = Q^-1 and m is the probe average of z_1 z_2.
    K = 64
    z = orc.probes(7, K, 2).astype(np.float64)
    m = (z[0] * z[1]).mean()
    S11, S22, S12 = a22 / det, a11 / det, lam / det
    s = orc.hutchinson(nbr, diag, lam, K, 7, 1e-15)
    assert np.allclose(s, [S11 + S12 * m, S22 + S12 * m], rtol=1e-10, atol=0)


def _tiny_system(orc, G=6, seed=0, lam=1.0, fill=0.6):
    rng = np.random.default_rng(seed)
    cells = [c for c in itertools.product(range(G), repeat=3) if rng.random() < fill]
    keys = np.sort(np.array([orc.morton_encode(*c) for c in cells], dtype=np.uint64))
    nbr, deg = orc.neighbours(G, keys)
    Lam = rng.uniform(0.5, 2.0, size=len(keys))
    diag = orc.precision_diag(Lam, deg, lam, 1e-6)
    return keys, nbr, deg, Lam, diag


def _dense_Q(orc, nbr, diag, lam):
    N = len(diag)
    Q = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        Q[:, j] = orc.apply_Q(nbr, diag, lam, e)
    return Q


def test_Q_symmetric_spd_and_quadratic_form(orc):
    """eq. (7)/(10): Q is symmetric, diagonally dominant with margin Lambda + eps,
    hence SPD with lambda_min >= eps, and x^T Q x equals
    sum Lambda x^2 + lam sum_edges (x_i - x_j)^2 + eps sum x^2."""
    lam, eps = 1.0, 1e-6
    keys, nbr, deg, Lam, diag = _tiny_system(orc, lam=lam)
    Q = _dense_Q(orc, nbr, diag, lam)
    assert np.array_equal(Q, Q.T)
    off = np.abs(Q).sum(1) - np.abs(np.diag(Q))
    assert np.allclose(np.diag(Q) - off, Lam + eps, rtol=1e-12)
    assert np.linalg.eigvalsh(Q).min() >= eps * (1 - 1e-9)
    bn = _brute_neighbours(6, keys, orc)
    edges = [(i, bn[i, s]) for i in range(len(keys)) for s in (1, 3, 5) if bn[i, s] >= 0]
    rng = np.random.default_rng(5)
    for _ in range(5):
        x = rng.standard_normal(len(keys))
        quad = (Lam * x * x).sum() + lam * sum((x[i] - x[j]) ** 2 for i, j in edges) + eps * (x * x).sum()
        assert math.isclose(x @ orc.apply_Q(nbr, diag, lam, x), quad, rel_tol=1e-12)


def test_pcg_diagonal_one_iteration(orc):
    """lam = 0 makes Q diagonal: Jacobi-PCG lands on b / diag in exactly one step."""
    keys, nbr, deg, Lam, diag0 = _tiny_system(orc, lam=0.0)
    diag = orc.precision_diag(Lam, deg, 0.0, 1e-6)
    b = np.random.default_rng(2).standard_normal(len(keys))
    x, rep = orc.pcg(nbr, diag, 0.0, b, 1e-12)
    assert rep["iters"] == 1 and rep["status"] == 0
    assert np.allclose(x, b / diag, rtol=1e-15, atol=0)


@pytest.mark.parametrize("lam", [1.0, 30.0])
def test_pcg_matches_cholesky(orc, lam):
    """Dense Cholesky solve of Q mu = b on a tiny band (scipy)."""
    keys, nbr, deg, Lam, diag = _tiny_system(orc, G=8, lam=lam)
    Q = _dense_Q(orc, nbr, diag, lam)
    b = np.random.default_rng(4).standard_normal(len(keys))
    ref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(Q), b)
    x, rep = orc.pcg(nbr, diag, lam, b, 1e-14)
    assert rep["status"] == 0 and rep["rel_res"] <= 1e-14
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-12


def test_pcg_zero_rhs_and_warm_start(orc):
    keys, nbr, deg, Lam, diag = _tiny_system(orc, lam=2.0)
    x, rep = orc.pcg(nbr, diag, 2.0, np.zeros(len(keys)), 1e-10)
    assert np.all(x == 0) and rep["iters"] == 0
    b = np.random.default_rng(9).standard_normal(len(keys))
    xs, _ = orc.pcg(nbr, diag, 2.0, b, 1e-14)
    x2, rep2 = orc.pcg(nbr, diag, 2.0, b, 1e-8, x0=xs)
    assert rep2["iters"] == 0 and np.array_equal(x2, xs)


# ----------------------------------------------------------------- Hutchinson
def test_probes_balanced_and_uncorrelated(orc):
    z = orc.probes(0, 16, 4000).astype(np.float64)
    assert set(np.unique(z)) == {-1.0, 1.0}
    assert np.abs(z.mean(0)).max() < 5 / math.sqrt(4000)
    C = (z.T @ z) / 4000
    assert np.abs(C - np.eye(16)).max() < 5 / math.sqrt(4000)


def test_hutchinson_exact_when_diagonal(orc):
    """lam = 0: z * (Q^-1 z) = diag(Q^-1) exactly for one Rademacher probe (eq. 12)."""
    keys, nbr, deg, Lam, _ = _tiny_system(orc, lam=0.0)
    diag = orc.precision_diag(Lam, deg, 0.0, 1e-6)
    s = orc.hutchinson(nbr, diag, 0.0, 1, 3, 1e-14)
    assert np.allclose(s, 1.0 / diag, rtol=1e-15, atol=0)


def test_hutchinson_error_law(orc):
    """Rademacher Hutchinson is unbiased and E[(s_i - S_ii)^2] = sum_{j != i} S_ij^2 / K
    with S = Q^-1; the RMS error falls as K^(-1/2)."""
    lam = 0.4
    keys, nbr, deg, Lam, diag = _tiny_system(orc, G=5, seed=1, lam=lam)
    S = np.linalg.inv(_dense_Q(orc, nbr, diag, lam))
    exact = np.diag(S)
    off2 = (S * S).sum(1) - exact ** 2
    for K in (1, 4, 16):
        errs = np.array([orc.hutchinson(nbr, diag, lam, K, seed, 1e-13) - exact
                         for seed in range(200)])
        mse = (errs ** 2).mean(0)
        pred = off2 / K
        assert abs(mse.sum() / pred.sum() - 1.0) < 0.15
        assert abs(errs.mean(0).sum()) < 4 * math.sqrt(pred.sum() / 200) * math.sqrt(len(exact))


# ----------------------------------------------------------------- NBV
def _full_band(orc, G):
    keys = np.sort(np.array([orc.morton_encode(*c) for c in itertools.product(range(G), repeat=3)],
                            dtype=np.uint64))
    return keys


def _sample_voxels(g, o, d, step=1e-4):
    """Ordered distinct voxels hit by points sampled densely along the ray."""
    G, h, org = g.G, g.h, np.array(g.origin[:])
    out = []
    dn = d / np.linalg.norm(d)
    for s in np.arange(0.0, 4.0, step):
        p = o + s * dn
        idx = np.floor((p - org) / h).astype(int)
        if np.all(idx >= 0) and np.all(idx < G):
            t = tuple(idx)
            if not out or out[-1] != t:
                out.append(t)
    return out


def test_nbv_ray_bruteforce(orc):
    """Constant variance, no surface: the score of a ray is the number of band voxels
    it crosses, compared with dense point sampling of the ray."""
    G, h = 8, 0.125
    g = orc.grid(G, h, (-0.5,) * 3, 0.5, 0.25)
    keys = _full_band(orc, G)
    N = len(keys)
    mu = np.ones(N)
    q = np.ones(N, dtype=np.int64)
    rng = np.random.default_rng(11)
    for _ in range(20):
        o = rng.normal(size=3)
        o = 1.5 * o / np.linalg.norm(o)
        target = rng.uniform(-0.3, 0.3, size=3)
        d = target - o
        sc, steps = orc.nbv_ray(g, keys, mu, q, o, d)
        vox = _sample_voxels(g, o, d)
        assert sc == len(vox) == steps
    # facing away: no voxel is crossed
    o = np.array([1.5, 0.0, 0.0])
    assert orc.nbv_ray(g, keys, mu, q, o, np.array([1.0, 0.1, 0.0]))[0] == 0


def test_nbv_ray_stops_at_surface(orc):
    """Accumulation runs up to and including the first voxel with mu <= 0."""
    G, h = 8, 0.125
    g = orc.grid(G, h, (-0.5,) * 3, 0.5, 0.25)
    keys = _full_band(orc, G)
    rng = np.random.default_rng(12)
    q = rng.integers(1, 1000, size=len(keys)).astype(np.int64)
    pos = {orc.morton_decode(k): n for n, k in enumerate(keys)}
    mu = np.ones(len(keys))
    for c, n in pos.items():
        if sum((x - 3.5) ** 2 for x in c) < 6.0:
            mu[n] = -1.0
    for _ in range(10):
        o = rng.normal(size=3)
        o = 1.5 * o / np.linalg.norm(o)
        d = rng.uniform(-0.1, 0.1, size=3) - o
        vox = _sample_voxels(g, o, d)
        want = 0
        for c in vox:
            want += int(q[pos[c]])
            if mu[pos[c]] <= 0:
                break
        assert orc.nbv_ray(g, keys, mu, q, o, d)[0] == want


def test_nbv_candidate_steps_sum_rays(orc):
    """A candidate's visit count is the sum of its pixel rays' walks, each pinned
    above against dense sampling; rays through pixel centres of the ray camera."""
    G, h = 8, 0.125
    g = orc.grid(G, h, (-0.5,) * 3, 0.5, 0.25)
    keys = _full_band(orc, G)
    mu = np.ones(len(keys))
    q = np.ones(len(keys), dtype=np.int64)
    cam = orc.cam(type("C", (), dict(width=6, height=5, fx=4.0, fy=4.0, cx=2.37, cy=1.91))())
    # camera near (0, 0, -1.5) looking along +z (OpenCV axes), off the grid's symmetry planes
    P = np.array([1.0, 0.0, 0.0, 0.013, 0.0, 1.0, 0.0, -0.021, 0.0, 0.0, 1.0, -1.5])
    total = 0
    for row in range(5):
        for col in range(6):
            d = np.array([(col - 2.37) / 4.0, (row - 1.91) / 4.0, 1.0])
            total += len(_sample_voxels(g, P[[3, 7, 11]], d))
    assert orc.nbv_walk_steps(g, cam, keys, mu, q, P[None, :])[0] == total > 0


def test_nbv_ties_lowest_index(orc):
    assert orc.nbv_argmax(np.array([3, 7, 7, 1], dtype=np.int64)) == 1
    assert orc.nbv_argmax(np.array([5, 5], dtype=np.int64)) == 0


def test_quantize_variance(orc):
    s = np.array([0.5, 1.0, 0.25, 0.0])
    assert list(orc.quantize_variance(s)) == [2 ** 31, 2 ** 32, 2 ** 30, 0]


# ----------------------------------------------------------------- features
def test_features_planar_wall(orc):
    """On the exact wall the TSDF gradient along z is -1 in the band interior,
    every voxel has one observation and TSDF/h is an integer."""
    G, h = 16, 2.0 ** -6
    z_plane = -G * h / 2 + 8.5 * h
    g, cm, P, depth = _wall(orc, G, h, z_plane, -1.0, 4 * h, 3 * h)
    td, wd = orc.tsdf_dense(g, cm, depth, P)
    keys, bt, bw = orc.band(g, td, wd)
    nbr, deg = orc.neighbours(G, keys)
    Lam, b, acc = orc.assemble(g, cm, depth, P, keys, with_acc=True)
    f = orc.features(1, h, bt, bw, nbr, deg, Lam, acc)
    assert np.all(f[:, 3] == 1.0)
    assert np.all(f[:, 0] == np.round(f[:, 0]))
    interior = (nbr[:, 4] >= 0) & (nbr[:, 5] >= 0)
    assert interior.sum() > 0 and np.all(f[interior, 11] == -1.0)
    assert np.all(f[:, 9] == 0.0) and np.all(f[:, 10] == 0.0)
    assert np.allclose(f[:, 4], bt / h)  # one view: mean y = TSDF
    assert np.all(f[:, 5] == 0.0)


def _rot(ax, ay, az):
    cx, sx, cy, sy, cz, sz = math.cos(ax), math.sin(ax), math.cos(ay), math.sin(ay), math.cos(az), math.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def _look_at_centre(R0, dist, jitter):
    """Camera-to-world pose (3x4, row-major) at dist from the origin whose optical
    axis (third column of R) points at the grid centre, before a small rotation."""
    R = R0
    o = -dist * R[:, 2] + jitter
    return np.concatenate([R, o[:, None]], axis=1).reshape(-1)


def _crossed_voxels(g, o, d):
    """Voxels the ray o + t d (t >= 0) passes through, in order: every time the ray
    crosses a grid plane is computed, the times are sorted, and each segment between
    consecutive crossings lies in the voxel holding its midpoint."""
    G, h, org = g.G, g.h, np.array(g.origin[:])
    ts = [0.0]
    for ax in range(3):
        if d[ax] != 0.0:
            ts.extend(((org[ax] + np.arange(G + 1) * h - o[ax]) / d[ax]).tolist())
    ts = np.unique(np.array([t for t in ts if t >= 0.0]))
    out = []
    for t0, t1 in zip(ts[:-1], ts[1:]):
        idx = np.floor((o + 0.5 * (t0 + t1) * d - org) / h).astype(int)
        if np.all(idx >= 0) and np.all(idx < G):
            out.append(tuple(int(i) for i in idx))
    return out


def _vr_setup(orc, seed):
    G, h = 8, 0.125
    g = orc.grid(G, h, (-0.5,) * 3, 0.5, 0.25)
    keys = _full_band(orc, G)
    rng = np.random.default_rng(seed)
    # variances with at most 20 significant bits, so s * s is exact and (s * s) / s == s
    s = rng.integers(1, 1 << 20, size=len(keys)).astype(np.float64) / 1024.0
    mu = np.ones(len(keys))
    for n, k in enumerate(keys):
        c = orc.morton_decode(int(k))
        if sum((x - 3.5) ** 2 for x in c) < 5.0:
            mu[n] = -1.0
    cam = orc.cam(type("C", (), dict(width=5, height=4, fx=3.0, fy=3.0, cx=1.93, cy=1.41))())
    poses = np.stack([_look_at_centre(_rot(*rng.uniform(-0.6, 0.6, 3)), 1.6, rng.uniform(-0.05, 0.05, 3))
                      for _ in range(4)])
    return g, keys, s, mu, cam, poses


def test_nbv_var_reduction_noiseless_equals_summed_variance(orc):
    """With a noiseless sensor (sigma = 0) one more observation removes all of a
    voxel's variance: s^2 / (s + 0) = s, so the expected-variance-reduction utility
    equals the summed-variance utility (pinned above by dense ray sampling)."""
    g, keys, s, mu, cam, poses = _vr_setup(orc, 21)
    q = orc.quantize_variance(s)
    want = orc.nbv_scores(g, cam, keys, mu, q, poses)
    got = orc.nbv_scores_var_reduction(g, cam, keys, mu, s, poses, noise=(0.0, 0.0, 0.4))
    assert np.all(want > 0)
    assert np.array_equal(got, want)


def test_nbv_var_reduction_depth_from_geometry(orc):
    """Depth-dependent sensor noise sigma(Z) = a + c (Z - z0)^2: the expected
    reduction at a voxel is s^2 / (s + sigma^2) with Z the voxel centre's depth
    along the candidate's optical axis (the rotation's third column), summed over
    the voxels each pixel ray crosses (from its sorted plane crossings) up to the
    first voxel with mu <= 0.  Each voxel's term may round differently by 1."""
    g, keys, s, mu, cam, poses = _vr_setup(orc, 22)
    a, c, z0 = 0.3, 2.0, 0.9
    smax = s.max()
    pos = {orc.morton_decode(int(k)): n for n, k in enumerate(keys)}
    got = orc.nbv_scores_var_reduction(g, cam, keys, mu, s, poses, noise=(a, c, z0))
    for ci, P in enumerate(poses):
        M = P.reshape(3, 4)
        R, o = M[:, :3], M[:, 3]
        want, nvox = 0, 0
        for row in range(cam.height):
            for col in range(cam.width):
                d = R @ np.array([(col - cam.cx) / cam.fx, (row - cam.cy) / cam.fy, 1.0])
                for vx in _crossed_voxels(g, o, d):
                    n = pos[vx]
                    centre = np.array(g.origin[:]) + (np.array(vx) + 0.5) * g.h
                    Z = float(R[:, 2] @ (centre - o))
                    sig = a + c * (Z - z0) ** 2
                    want += int(np.rint(s[n] ** 2 / (s[n] + sig ** 2) / smax * 2.0 ** 32))
                    nvox += 1
                    if mu[n] <= 0:
                        break
        assert nvox > 20
        assert abs(int(got[ci]) - want) <= nvox, (ci, got[ci], want)
    # the noise model matters: a noiseless sensor gives strictly larger utilities
    assert np.all(orc.nbv_scores_var_reduction(g, cam, keys, mu, s, poses, noise=(0.0, 0.0, z0)) > got)


def test_oracle_threads_do_not_change_results():
    """The oracle's OpenMP loops (dense TSDF, neighbours, assembly, one solve per
    probe, one NBV candidate per iteration) give the same bits on 1 thread and
    on several."""
    import oracle as O
    from synth import make_workload
    wl = make_workload("tiny")
    cands = wl.candidates()[:24]
    nthreads = max(2, min(8, O.max_threads()))
    runs = []
    try:
        for t in (1, nthreads):
            O.set_threads(t)
            ref = O.full_pipeline(wl, with_acc=True)
            mu, _ = O.pcg(ref["nbr"], ref["diag"], wl.lam, ref["rhs"], 1e-10)
            s = O.hutchinson(ref["nbr"], ref["diag"], wl.lam, 8, 3, 1e-10)
            q = O.quantize_variance(s)
            sc, st = O.nbv_scores_steps(ref["grid"], O.cam(wl.ray_cam), ref["keys"], mu, q, cands)
            runs.append((ref, mu, s, sc, st))
    finally:
        O.set_threads(O.max_threads())
    (r1, mu1, s1, sc1, st1), (r2, mu2, s2, sc2, st2) = runs
    for k in ("tsdf_dense", "w_dense", "keys", "tsdf", "w", "nbr", "deg", "Lambda", "b", "diag", "rhs", "acc"):
        assert np.array_equal(r1[k], r2[k]), k
    assert np.array_equal(mu1, mu2) and np.array_equal(s1, s2)
    assert np.array_equal(sc1, sc2) and np.array_equal(st1, st2)
