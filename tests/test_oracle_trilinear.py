"""Pins of the oracle's trilinear observation rows (Sec. 3.2, eqs. 2-5) and of
the 27-point system they give (eqs. 7, 10-12), each against something other
than the oracle's own arithmetic:

* geometry: every kept sample, rebuilt from its 8 corner weights (trilinear
  interpolation reproduces linear functions, here the position), projects
  onto the centre of its own pixel (t, row, col) at camera depth D + s h, and
  its y is clamp(D - Z, -tau, tau) of that pixel's depth D;
* the cell-grouped assembly against a dense A^T W A and A^T W y built with a
  numpy matrix product from the explicit sample rows;
* exact symmetry and positive definiteness (Cholesky) of Q, and the quadratic
  form sum_i w_i (a_i.x)^2 + lam sum_E (x_u - x_v)^2 + eps |x|^2;
* the 27-point PCG against a dense solve, and the Hutchinson estimate against
  the same probes applied to the dense inverse.
"""
import numpy as np
import pytest

import oracle as O
from synth import make_workload


def _corner(q):
    return np.array([q & 1, (q >> 1) & 1, q >> 2])


@pytest.fixture(scope="module")
def tiny():
    wl = make_workload("tiny")
    ref = O.full_pipeline(wl)
    S = int(round(wl.tau / wl.h))
    tri = O.tri_assemble(ref["grid"], ref["cam"], wl.depth, wl.poses, ref["keys"], ref["deg"], ref["tsdf"], S,
                         wl.lam, wl.eps, wl.lam_b, noise=wl.noise)
    base, a, y, w, tcrs = O.tri_samples(ref["grid"], ref["cam"], wl.depth, wl.poses, ref["keys"], S,
                                        noise=wl.noise)
    return wl, ref, S, tri, (base, a, y, w, tcrs)


def _dense_A(ref, base, a):
    keys = ref["keys"]
    index = {int(k): i for i, k in enumerate(keys)}
    A = np.zeros((len(a), len(keys)))
    for q in range(8):
        c = base + _corner(q)
        cols = np.array([index[O.morton_encode(int(i), int(j), int(k))] for i, j, k in c])
        A[np.arange(len(a)), cols] += a[:, q]
    return A


def _dense_Q(tri):
    N = len(tri["diag"])
    Q = np.diag(tri["diag"])
    for slot in range(26):
        u = tri["nb26"][:, slot]
        m = u >= 0
        Q[np.nonzero(m)[0], u[m]] += tri["off"][m, slot]
    return Q


def test_tri_samples_lie_on_pixel_rays(tiny):
    wl, ref, S, tri, (base, a, y, w, tcrs) = tiny
    assert len(a) == tri["samples"] > 1000
    assert np.all(a >= 0.0) and np.allclose(a.sum(axis=1), 1.0, rtol=0, atol=1e-14)
    # sample points from the corner weights (voxel centres at (i + 1/2) h)
    centres = np.stack([(base + _corner(q) + 0.5) * wl.h + np.asarray(wl.origin) for q in range(8)], axis=1)
    p = np.einsum("nq,nqd->nd", a, centres)
    cam = wl.cam
    t, row, col, s = tcrs.T
    P = np.asarray(wl.poses).reshape(-1, 3, 4)[t]
    Xc = np.einsum("nda,nd->na", P[:, :, :3], p - P[:, :, 3])  # R^T (p - t) per sample
    u = cam.fx * Xc[:, 0] / Xc[:, 2] + cam.cx
    v = cam.fy * Xc[:, 1] / Xc[:, 2] + cam.cy
    assert np.all(np.abs(u - col) < 1e-7) and np.all(np.abs(v - row) < 1e-7)
    D = np.asarray(wl.depth)[t, row, col].astype(np.float64)
    assert np.all(np.abs(Xc[:, 2] - (D + s * wl.h)) < 1e-9)
    assert np.all(np.abs(np.clip(D - Xc[:, 2], -wl.tau, wl.tau) - y) < 1e-9)
    assert np.all(np.abs(s) <= S)
    assert np.all(np.abs(y) <= wl.tau) and np.all(w > 0)


def _morton(i, j, k):
    key = np.zeros(np.shape(i), dtype=np.uint64)
    for b in range(21):
        for axis, c in enumerate((i, j, k)):
            key |= ((np.asarray(c, dtype=np.int64) >> b) & 1).astype(np.uint64) << np.uint64(3 * b + axis)
    return key


def test_tri_sample_set_brute_force(tiny):
    """Every candidate (t, row, col, s) enumerated with numpy: the samples whose
    8 surrounding voxel centres are band voxels are exactly the oracle's."""
    wl, ref, S, tri, (base, a, y, w, tcrs) = tiny
    cam, h, G = wl.cam, wl.h, wl.G
    band = set(int(k) for k in ref["keys"])
    rows, cols = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    ra = (cols - cam.cx) / cam.fx
    rb = (rows - cam.cy) / cam.fy
    want = set()
    for t in range(wl.T):
        P = np.asarray(wl.poses[t]).reshape(3, 4)
        D = np.asarray(wl.depth[t], dtype=np.float64)
        for s in range(-S, S + 1):
            z = D + s * h
            ok = (D > 0) & np.isfinite(D) & (z > 0)
            fl = []
            for r in range(3):
                x = P[r, 3] + z * ((P[r, 0] * ra + P[r, 1] * rb) + P[r, 2])
                f = np.floor((x - wl.origin[r]) / h - 0.5)
                ok &= (f >= 0) & (f + 1 <= G - 1)
                fl.append(np.where(ok, f, 0).astype(np.int64))
            for q in range(8):
                c = _corner(q)
                keys = _morton(fl[0] + c[0], fl[1] + c[1], fl[2] + c[2])
                inb = np.fromiter((int(k) in band for k in keys.ravel()), bool, keys.size).reshape(keys.shape)
                ok &= inb
            for rr, cc in zip(*np.nonzero(ok)):
                want.add((t, int(rr), int(cc), s))
    got = set(map(tuple, tcrs.tolist()))
    assert got == want and len(got) == len(tcrs)


def test_tri_assembly_matches_dense_product(tiny):
    wl, ref, S, tri, (base, a, y, w, tcrs) = tiny
    A = _dense_A(ref, base, a)
    AtWA = A.T @ (w[:, None] * A)
    AtWy = A.T @ (w * y)
    scale = np.abs(AtWA).max()
    assert np.allclose(tri["Lambda"], np.diag(AtWA), rtol=1e-12, atol=1e-12 * scale)
    assert np.allclose(tri["b"], AtWy, rtol=1e-12, atol=1e-12 * np.abs(AtWy).max())
    # couplings: A^T W A off the diagonal, minus lam on the band's face edges
    N = len(ref["keys"])
    L = np.zeros((N, N))
    for t in range(6):
        u = ref["nbr"][:, t]
        m = u >= 0
        L[np.nonzero(m)[0], u[m]] = -wl.lam
    Qd = _dense_Q(tri)
    want = AtWA + L
    np.fill_diagonal(want, 0.0)
    got = Qd.copy()
    np.fill_diagonal(got, 0.0)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * scale)
    assert np.array_equal(tri["diag"], O.precision_diag(tri["Lambda"], ref["deg"], wl.lam, wl.eps, wl.lam_b))


def test_tri_neighbour_slots_brute_force(tiny):
    wl, ref, S, tri, _ = tiny
    keys = ref["keys"]
    index = {int(k): i for i, k in enumerate(keys)}
    rng = np.random.default_rng(3)
    for v in rng.choice(len(keys), size=300, replace=False):
        i, j, k = O.morton_decode(int(keys[v]))
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    slot = O.tri_slot(dx, dy, dz)
                    if slot < 0:
                        continue
                    ni, nj, nk = i + dx, j + dy, k + dz
                    inside = 0 <= min(ni, nj, nk) and max(ni, nj, nk) < wl.G
                    want = index.get(O.morton_encode(ni, nj, nk), -1) if inside else -1
                    assert tri["nb26"][v, slot] == want


def test_tri_Q_symmetric_spd_and_quadratic_form(tiny):
    wl, ref, S, tri, (base, a, y, w, tcrs) = tiny
    Q = _dense_Q(tri)
    assert np.array_equal(Q, Q.T)  # the shared cell sums make Q exactly symmetric
    np.linalg.cholesky(Q)  # raises unless positive definite
    A = _dense_A(ref, base, a)
    rng = np.random.default_rng(5)
    nbr = ref["nbr"]
    for _ in range(3):
        x = rng.standard_normal(len(ref["keys"]))
        edges = sum(((x[nbr[:, t] >= 0] - x[nbr[nbr[:, t] >= 0, t]]) ** 2).sum() for t in (1, 3, 5))
        want = (w * (A @ x) ** 2).sum() + wl.lam * edges + wl.eps * (x * x).sum()
        if wl.lam_b:
            want += wl.lam_b * (x[ref["deg"] < 6] ** 2).sum()
        assert np.isclose(x @ Q @ x, want, rtol=1e-11)
        assert np.allclose(O.apply_Q27(tri["diag"], tri["off"], tri["nb26"], x), Q @ x, rtol=1e-12,
                           atol=1e-12 * np.abs(Q @ x).max())


def test_pcg27_matches_dense_solve(tiny):
    wl, ref, S, tri, _ = tiny
    Q = _dense_Q(tri)
    mu_dense = np.linalg.solve(Q, tri["rhs"])
    mu, rep = O.pcg27(tri["diag"], tri["off"], tri["nb26"], tri["rhs"], 1e-13)
    assert rep["status"] == 0 and rep["rel_res"] <= 1e-13
    assert np.linalg.norm(mu - mu_dense) <= 1e-11 * np.linalg.norm(mu_dense)


def test_hutchinson27_matches_dense_inverse(tiny):
    wl, ref, S, tri, _ = tiny
    Q = _dense_Q(tri)
    K = 4
    Z = O.probes(0, K, len(tri["diag"])).astype(np.float64)
    U = np.linalg.solve(Q, Z)
    want = (Z * U).sum(axis=1) / K
    s = O.hutchinson27(tri["diag"], tri["off"], tri["nb26"], K, 0, 1e-13)
    assert np.linalg.norm(s - want) <= 1e-10 * np.linalg.norm(want)
