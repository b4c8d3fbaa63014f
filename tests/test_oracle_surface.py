"""Pins of the oracle's surface extraction (Algorithm 1 step 7: marching
tetrahedra over the band) and of the geometry metrics (eq. 14), against
closed forms, topology and an independent library:

* a sphere field gives a closed, consistently oriented 2-manifold (every edge
  in exactly two triangles, Euler characteristic V - E + F = 2, every normal
  pointing away from the centre) whose vertices are within the linear
  interpolation bound of the sphere;
* an axis-aligned plane field gives vertices exactly on the plane and a total
  triangle area equal to the plane's cross-section of the voxel-centre hull;
* a tilted plane gives vertices on the plane, and every interior edge in two
  triangles;
* nearest-point distances equal scipy's k-d tree query; the metrics of a set
  against itself are exact (CD 0, F 1).
"""
import numpy as np
import pytest

import oracle as O


def _full_grid(G, h):
    keys = np.array(sorted(O.morton_encode(i, j, k) for i in range(G) for j in range(G) for k in range(G)),
                    dtype=np.uint64)
    ijk = np.array([O.morton_decode(int(k)) for k in keys], dtype=np.int64)
    origin = -0.5 * G * h
    return O.grid(G, h, (origin,) * 3, 5 * h, 1e9), keys, (ijk + 0.5) * h + origin


def _edges(tris):
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    return np.sort(e, axis=1)


def _normals(v, t):
    return np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])


@pytest.mark.parametrize("G,r", [(16, 0.3), (24, 0.37)])
def test_sphere_mesh_closed_oriented_and_close(G, r):
    h = 1.0 / G
    g, keys, x = _full_grid(G, h)
    centre = np.array([0.013, -0.021, 0.008])
    mu = np.linalg.norm(x - centre, axis=1) - r
    v, t = O.extract_surface(g, keys, mu)
    assert len(t) > 100
    edges = _edges(t)
    uniq, counts = np.unique(edges, axis=0, return_counts=True)
    assert np.all(counts == 2)  # closed manifold
    assert len(v) - len(uniq) + len(t) == 2  # Euler characteristic of a sphere
    assert np.all(np.isin(np.arange(len(v)), t))  # every vertex used
    c = v[t].mean(axis=1)
    assert np.all(np.einsum("ij,ij->i", _normals(v, t), c - centre) > 0)  # outward
    # linear interpolation of |x - c| - r along an edge of length l <= sqrt(3) h
    ell = np.sqrt(3.0) * h
    bound = ell * ell / (8.0 * (r - ell))
    assert np.abs(np.linalg.norm(v - centre, axis=1) - r).max() <= bound


def test_axis_plane_exact_area():
    G = 12
    h = 1.0 / G
    g, keys, x = _full_grid(G, h)
    c = 0.0371
    mu = x[:, 2] - c
    v, t = O.extract_surface(g, keys, mu)
    assert np.abs(v[:, 2] - c).max() <= 1e-15
    area = 0.5 * np.linalg.norm(_normals(v, t), axis=1).sum()
    assert abs(area - ((G - 1) * h) ** 2) <= 1e-12
    assert np.all(_normals(v, t)[:, 2] > 0)  # normals towards mu > 0 (+z)


def test_tilted_plane_on_plane_and_watertight_inside():
    G = 14
    h = 1.0 / G
    g, keys, x = _full_grid(G, h)
    n = np.array([0.3, -0.5, 0.81])
    n = n / np.linalg.norm(n)
    c = 0.05
    mu = x @ n - c
    v, t = O.extract_surface(g, keys, mu)
    assert np.abs(v @ n - c).max() <= 1e-14
    lo, hi = x.min(axis=0), x.max(axis=0)
    edges, counts = np.unique(_edges(t), axis=0, return_counts=True)
    a, b = v[edges[:, 0]], v[edges[:, 1]]
    on_hull = np.zeros(len(edges), dtype=bool)
    for ax in range(3):
        for bound in (lo[ax], hi[ax]):
            on_hull |= (np.abs(a[:, ax] - bound) < 1e-12) & (np.abs(b[:, ax] - bound) < 1e-12)
    assert np.all(counts[~on_hull] == 2) and np.all(counts[on_hull] == 1)


def test_band_subset_mesh_uses_only_band_cubes():
    """On a band (not the full grid) only cubes with 8 band corners give
    triangles; a vertex needs both edge ends in the band."""
    G = 16
    h = 1.0 / G
    g, keys, x = _full_grid(G, h)
    mu = np.linalg.norm(x, axis=1) - 0.3
    keep = np.abs(mu) <= 1.5 * h
    v, t = O.extract_surface(g, keys[keep], mu[keep])
    vf, tf = O.extract_surface(g, keys, mu)
    assert 0 < len(t) <= len(tf) and 0 < len(v) <= len(vf)
    assert np.abs(np.linalg.norm(v, axis=1) - 0.3).max() <= 0.02


def test_nn_distances_match_kdtree_and_metrics_identities():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(11)
    a = rng.standard_normal((700, 3))
    b = rng.standard_normal((900, 3)) * 1.3 + 0.1
    d = O.nn_dist2(a, b)
    dk, _ = cKDTree(b).query(a)
    assert np.allclose(d, dk * dk, rtol=1e-14, atol=0)
    m, dp, dg = O.surface_metrics(a, a, [0.01, 0.1])
    assert m["chamfer"] == 0.0 and m["accuracy"] == 0.0 and m["completeness"] == 0.0
    assert m["fscore"] == [1.0, 1.0]
    m, dp, dg = O.surface_metrics(a, b, [0.2])
    want_cd = np.mean(cKDTree(b).query(a)[0] ** 2) + np.mean(cKDTree(a).query(b)[0] ** 2)
    assert np.isclose(m["chamfer"], want_cd, rtol=1e-12)
