"""ctypes shim over the FP64 CPU oracle (oracle.c) plus the numpy MLP oracle.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  Arrays go in and
come out as numpy; every routine is documented where it is defined in C.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_F = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_I64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_U64 = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


class Grid(C.Structure):
    _fields_ = [("G", C.c_int32), ("h", C.c_double), ("origin", C.c_double * 3),
                ("tau", C.c_double), ("band", C.c_double)]


class Cam(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double),
                ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class Noise(C.Structure):
    _fields_ = [("a", C.c_double), ("c", C.c_double), ("z0", C.c_double),
                ("sigma2_pose", C.POINTER(C.c_double)), ("sigma2_model", C.c_double)]


class Utility(C.Structure):
    _fields_ = [("utility", C.c_int32), ("a", C.c_double), ("c", C.c_double), ("z0", C.c_double),
                ("s", C.c_void_p), ("smax", C.c_double)]


class Report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("rel_res", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_max_threads.restype = C.c_int32
        L.orc_morton_encode.restype = C.c_uint64
        L.orc_morton_encode.argtypes = [C.c_int32] * 3
        L.orc_morton_decode.argtypes = [C.c_uint64] + [C.POINTER(C.c_int32)] * 3
        L.orc_tsdf_voxel.argtypes = [C.POINTER(Grid), C.POINTER(Cam), C.c_int32, _F, _D, C.c_int32,
                                     C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int32)]
        L.orc_tsdf_dense.argtypes = [C.POINTER(Grid), C.POINTER(Cam), C.c_int32, _F, _D, _D, _I32]
        L.orc_tsdf_points.argtypes = [C.POINTER(Grid), C.POINTER(Cam), C.c_int32, _F, _D, C.c_int64,
                                      _I32, _D, _I32]
        L.orc_band.restype = C.c_int64
        L.orc_band.argtypes = [C.POINTER(Grid), _D, _I32, C.c_int64, C.c_void_p, C.c_void_p,
                               C.c_void_p]
        L.orc_neighbours.argtypes = [C.c_int32, _U64, C.c_int64, _I32, _I32]
        L.orc_assemble.argtypes = [C.POINTER(Grid), C.POINTER(Cam), C.c_int32, _F, _D,
                                   C.POINTER(Noise), _U64, C.c_int64, _D, _D, C.c_void_p]
        L.orc_precision_diag.argtypes = [C.c_int64, _D, _I32, C.c_double, C.c_double, C.c_double, _D]
        L.orc_anchor_rhs.argtypes = [C.c_int64, _D, _I32, _D, C.c_double, _D]
        L.orc_apply_Q.argtypes = [C.c_int64, _I32, _D, C.c_double, _D, _D]
        L.orc_pcg.argtypes = [C.c_int64, _I32, _D, C.c_double, _D, C.c_void_p, C.c_double,
                              C.c_int32, _D, C.POINTER(Report)]
        L.orc_splitmix_output.restype = C.c_uint64
        L.orc_splitmix_output.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_probe_sign.restype = C.c_int32
        L.orc_probe_sign.argtypes = [C.c_uint64, C.c_int32, C.c_int64]
        L.orc_hutchinson.argtypes = [C.c_int64, _I32, _D, C.c_double, C.c_int32, C.c_uint64,
                                     C.c_double, C.c_int32, _D, C.c_void_p]
        L.orc_quantize_variance.argtypes = [C.c_int64, _D, _I64]
        L.orc_nbv_ray.restype = C.c_int64
        L.orc_nbv_ray.argtypes = [C.POINTER(Grid), _U64, C.c_int64, _D, _I64, _D, _D, C.c_void_p]
        L.orc_nbv_candidate.restype = C.c_int64
        L.orc_nbv_candidate.argtypes = [C.POINTER(Grid), C.POINTER(Cam), _U64, C.c_int64, _D, _I64,
                                        _D]
        L.orc_nbv_candidate_steps.restype = C.c_int64
        L.orc_nbv_candidate_steps.argtypes = L.orc_nbv_candidate.argtypes
        L.orc_nbv_candidate_u.restype = C.c_int64
        L.orc_nbv_candidate_u.argtypes = [C.POINTER(Grid), C.POINTER(Cam), _U64, C.c_int64, _D,
                                          _I64, C.POINTER(Utility), _D]
        L.orc_nbv_scores.argtypes = [C.POINTER(Grid), C.POINTER(Cam), _U64, C.c_int64, _D, _I64, C.c_void_p,
                                     C.c_int32, _D, _I64, C.c_void_p]
        L.orc_pred_depth.argtypes = [C.POINTER(Grid), C.POINTER(Cam), _U64, C.c_int64, _D, _D, _F]
        L.orc_nbv_argmax.restype = C.c_int32
        L.orc_nbv_argmax.argtypes = [C.c_int32, _I64]
        L.orc_features.argtypes = [C.c_int64, C.c_int32, C.c_double, _D, _I32, _I32, _I32, _D, _D,
                                   _D]
        L.orc_tri_slot.restype = C.c_int32
        L.orc_tri_slot.argtypes = [C.c_int32] * 3
        L.orc_tri_sample_list.restype = C.c_int64
        L.orc_tri_sample_list.argtypes = [C.POINTER(Grid), C.POINTER(Cam), C.c_int32, _F, _D, C.POINTER(Noise),
                                          C.c_int32, _U64, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_tri_assemble.restype = C.c_int64
        L.orc_tri_assemble.argtypes = [C.POINTER(Grid), C.POINTER(Cam), C.c_int32, _F, _D, C.POINTER(Noise),
                                       C.c_int32, _U64, C.c_int64, _I32, _D, C.c_double, C.c_double,
                                       C.c_double, _D, _D, _D, _D, _D, _I32, C.POINTER(C.c_int64)]
        L.orc_apply_Q27.argtypes = [C.c_int64, _D, _D, _I32, _D, _D]
        L.orc_pcg27.argtypes = [C.c_int64, _D, _D, _I32, _D, C.c_void_p, C.c_double, C.c_int32, _D,
                                C.POINTER(Report)]
        L.orc_hutchinson27.argtypes = [C.c_int64, _D, _D, _I32, C.c_int32, C.c_uint64, C.c_double, C.c_int32,
                                       _D, C.c_void_p]
        L.orc_surf_dir.restype = C.c_int32
        L.orc_surf_dir.argtypes = [C.c_int32] * 3
        L.orc_extract_surface.argtypes = [C.POINTER(Grid), _U64, C.c_int64, _D, C.c_double, C.c_int64, C.c_int64,
                                          C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.orc_nn_dist2.argtypes = [_D, C.c_int64, _D, C.c_int64, _D]
        _lib = L
    return _lib


# ---------------------------------------------------------------- helpers
def grid(G, h, origin, tau, band) -> Grid:
    g = Grid()
    g.G, g.h, g.tau, g.band = int(G), float(h), float(tau), float(band)
    for a in range(3):
        g.origin[a] = float(origin[a])
    return g


def cam(c) -> Cam:
    out = Cam()
    out.width, out.height = int(c.width), int(c.height)
    out.fx, out.fy, out.cx, out.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
    return out


def grid_of(w) -> Grid:
    """Oracle grid for a synthetic workload object (G, h, origin, tau, band)."""
    return grid(w.G, w.h, w.origin, w.tau, w.band)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (every result is independent of it)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def morton_encode(i, j, k) -> int:
    return int(lib().orc_morton_encode(int(i), int(j), int(k)))


def morton_decode(key):
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    lib().orc_morton_decode(C.c_uint64(int(key)), C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def tsdf_voxel(g: Grid, cm: Cam, depth, c2w, i, j, k):
    t, w = C.c_double(), C.c_int32()
    depth = _c(depth, np.float32)
    lib().orc_tsdf_voxel(C.byref(g), C.byref(cm), depth.shape[0], depth, _c(c2w, np.float64),
                         int(i), int(j), int(k), C.byref(t), C.byref(w))
    return t.value, w.value


def tsdf_points(g: Grid, cm: Cam, depth, c2w, ijk):
    """Coarse TSDF and weight of the voxels ijk [n][3]."""
    depth = _c(depth, np.float32)
    ijk = _c(ijk, np.int32).reshape(-1, 3)
    n = ijk.shape[0]
    t = np.zeros(max(n, 1), dtype=np.float64)
    w = np.zeros(max(n, 1), dtype=np.int32)
    lib().orc_tsdf_points(C.byref(g), C.byref(cm), depth.shape[0], depth, _c(c2w, np.float64), n, ijk, t, w)
    return t[:n], w[:n]


def tsdf_dense(g: Grid, cm: Cam, depth, c2w):
    """Dense coarse TSDF and weights, arrays indexed [k][j][i]."""
    depth = _c(depth, np.float32)
    G = g.G
    tsdf = np.zeros(G * G * G, dtype=np.float64)
    w = np.zeros(G * G * G, dtype=np.int32)
    lib().orc_tsdf_dense(C.byref(g), C.byref(cm), depth.shape[0], depth, _c(c2w, np.float64), tsdf, w)
    return tsdf.reshape(G, G, G), w.reshape(G, G, G)


def band(g: Grid, tsdf_dense, w_dense):
    t = _c(tsdf_dense, np.float64).reshape(-1)
    w = _c(w_dense, np.int32).reshape(-1)
    n = lib().orc_band(C.byref(g), t, w, 0, None, None, None)
    keys = np.zeros(max(n, 1), dtype=np.uint64)
    bt = np.zeros(max(n, 1), dtype=np.float64)
    bw = np.zeros(max(n, 1), dtype=np.int32)
    lib().orc_band(C.byref(g), t, w, n, keys.ctypes.data, bt.ctypes.data, bw.ctypes.data)
    return keys[:n], bt[:n], bw[:n]


def neighbours(G, keys):
    keys = _c(keys, np.uint64)
    N = keys.shape[0]
    nbr = np.zeros((max(N, 1), 6), dtype=np.int32)
    deg = np.zeros(max(N, 1), dtype=np.int32)
    lib().orc_neighbours(int(G), keys, N, nbr, deg)
    return nbr[:N], deg[:N]


def assemble(g: Grid, cm: Cam, depth, c2w, keys, noise=(0.0012, 0.0019, 0.4), sigma2_pose=None,
             sigma2_model=0.0, with_acc=False):
    depth = _c(depth, np.float32)
    keys = _c(keys, np.uint64)
    N = keys.shape[0]
    nz = Noise()
    nz.a, nz.c, nz.z0 = (float(v) for v in noise)
    nz.sigma2_model = float(sigma2_model)
    pose_arr = None
    if sigma2_pose is not None:
        pose_arr = _c(sigma2_pose, np.float64)
        nz.sigma2_pose = pose_arr.ctypes.data_as(C.POINTER(C.c_double))
    Lam = np.zeros(max(N, 1), dtype=np.float64)
    b = np.zeros(max(N, 1), dtype=np.float64)
    acc = np.zeros((max(N, 1), 5), dtype=np.float64) if with_acc else None
    lib().orc_assemble(C.byref(g), C.byref(cm), depth.shape[0], depth, _c(c2w, np.float64),
                       C.byref(nz), keys, N, Lam, b, acc.ctypes.data if with_acc else None)
    if with_acc:
        return Lam[:N], b[:N], acc[:N]
    return Lam[:N], b[:N]


def precision_diag(Lam, deg, lam, eps, lam_b=0.0):
    Lam = _c(Lam, np.float64)
    out = np.zeros(max(Lam.shape[0], 1), dtype=np.float64)
    lib().orc_precision_diag(Lam.shape[0], Lam, _c(deg, np.int32), float(lam), float(eps),
                             float(lam_b), out)
    return out[:Lam.shape[0]]


def anchor_rhs(b, deg, tsdf, lam_b):
    b = _c(b, np.float64)
    out = np.zeros(max(b.shape[0], 1), dtype=np.float64)
    lib().orc_anchor_rhs(b.shape[0], b, _c(deg, np.int32), _c(tsdf, np.float64), float(lam_b), out)
    return out[:b.shape[0]]


def apply_Q(nbr, diag, lam, p):
    p = _c(p, np.float64)
    q = np.zeros(max(p.shape[0], 1), dtype=np.float64)
    lib().orc_apply_Q(p.shape[0], _c(nbr, np.int32), _c(diag, np.float64), float(lam), p, q)
    return q[:p.shape[0]]


def pcg(nbr, diag, lam, rhs, tol, max_iter=10000, x0=None):
    rhs = _c(rhs, np.float64)
    N = rhs.shape[0]
    x = np.zeros(max(N, 1), dtype=np.float64)
    rep = Report()
    x0a = _c(x0, np.float64) if x0 is not None else None
    lib().orc_pcg(N, _c(nbr, np.int32), _c(diag, np.float64), float(lam), rhs,
                  x0a.ctypes.data if x0a is not None else None, float(tol), int(max_iter), x,
                  C.byref(rep))
    return x[:N], {"iters": rep.iters, "status": rep.status, "rel_res": rep.rel_res}


def splitmix_output(start, n) -> int:
    return int(lib().orc_splitmix_output(C.c_uint64(int(start)), C.c_uint64(int(n))))


def probe_sign(seed, k, i) -> int:
    return int(lib().orc_probe_sign(C.c_uint64(int(seed)), int(k), int(i)))


def probes(seed, K, N):
    """Rademacher probe matrix z[N][K] (int8) from the oracle's generator."""
    L = lib()
    z = np.empty((N, K), dtype=np.int8)
    for k in range(K):
        for i in range(N):
            z[i, k] = L.orc_probe_sign(C.c_uint64(int(seed)), k, i)
    return z


def hutchinson(nbr, diag, lam, K, seed, tol, max_iter=10000, with_iters=False):
    diag = _c(diag, np.float64)
    N = diag.shape[0]
    s = np.zeros(max(N, 1), dtype=np.float64)
    its = np.zeros(max(K, 1), dtype=np.int32)
    lib().orc_hutchinson(N, _c(nbr, np.int32), diag, float(lam), int(K), C.c_uint64(int(seed)),
                         float(tol), int(max_iter), s, its.ctypes.data)
    if with_iters:
        return s[:N], its[:K]
    return s[:N]


def _noise(noise, sigma2_pose=None, sigma2_model=0.0):
    nz = Noise()
    nz.a, nz.c, nz.z0 = (float(v) for v in noise)
    nz.sigma2_model = float(sigma2_model)
    keep = None
    if sigma2_pose is not None:
        keep = _c(sigma2_pose, np.float64)
        nz.sigma2_pose = keep.ctypes.data_as(C.POINTER(C.c_double))
    return nz, keep


def tri_slot(dx, dy, dz) -> int:
    return int(lib().orc_tri_slot(dx, dy, dz))


def tri_samples(g: Grid, cm: Cam, depth, c2w, keys, S, noise=(0.0012, 0.0019, 0.4), sigma2_pose=None,
                sigma2_model=0.0):
    """Kept trilinear samples in (cell, id) order: base[n][3], a[n][8], y[n], w[n] and
    (t, row, col, s)[n][4]."""
    depth = _c(depth, np.float32)
    keys = _c(keys, np.uint64)
    c2w = _c(c2w, np.float64)
    nz, keep = _noise(noise, sigma2_pose, sigma2_model)
    L = lib()
    n = L.orc_tri_sample_list(C.byref(g), C.byref(cm), depth.shape[0], depth, c2w, C.byref(nz), int(S), keys,
                              keys.shape[0], 0, None, None, None, None, None)
    base = np.zeros((max(n, 1), 3), dtype=np.int32)
    a = np.zeros((max(n, 1), 8), dtype=np.float64)
    y = np.zeros(max(n, 1), dtype=np.float64)
    w = np.zeros(max(n, 1), dtype=np.float64)
    tcrs = np.zeros((max(n, 1), 4), dtype=np.int32)
    L.orc_tri_sample_list(C.byref(g), C.byref(cm), depth.shape[0], depth, c2w, C.byref(nz), int(S), keys,
                          keys.shape[0], n, base.ctypes.data, a.ctypes.data, y.ctypes.data, w.ctypes.data,
                          tcrs.ctypes.data)
    return base[:n], a[:n], y[:n], w[:n], tcrs[:n]


def tri_assemble(g: Grid, cm: Cam, depth, c2w, keys, deg, tsdf, S, lam, eps, lam_b=0.0,
                 noise=(0.0012, 0.0019, 0.4), sigma2_pose=None, sigma2_model=0.0):
    """Trilinear system: dict of Lambda, b, rhs, diag [N], off, nb26 [N][26], samples, cells."""
    depth = _c(depth, np.float32)
    keys = _c(keys, np.uint64)
    N = keys.shape[0]
    nz, keep = _noise(noise, sigma2_pose, sigma2_model)
    M = max(N, 1)
    out = {k: np.zeros(M, dtype=np.float64) for k in ("Lambda", "b", "rhs", "diag")}
    off = np.zeros((M, 26), dtype=np.float64)
    nb26 = np.full((M, 26), -1, dtype=np.int32)
    ncell = C.c_int64(0)
    n = lib().orc_tri_assemble(C.byref(g), C.byref(cm), depth.shape[0], depth, _c(c2w, np.float64),
                               C.byref(nz), int(S), keys, N, _c(deg, np.int32), _c(tsdf, np.float64),
                               float(lam), float(eps), float(lam_b), out["Lambda"], out["b"], out["rhs"],
                               out["diag"], off, nb26, C.byref(ncell))
    res = {k: v[:N] for k, v in out.items()}
    res.update(off=off[:N], nb26=nb26[:N], samples=int(n), cells=int(ncell.value))
    return res


def apply_Q27(diag, off, nb26, p):
    p = _c(p, np.float64)
    q = np.zeros(max(p.shape[0], 1), dtype=np.float64)
    lib().orc_apply_Q27(p.shape[0], _c(diag, np.float64), _c(off, np.float64), _c(nb26, np.int32), p, q)
    return q[:p.shape[0]]


def pcg27(diag, off, nb26, rhs, tol, max_iter=10000, x0=None):
    rhs = _c(rhs, np.float64)
    N = rhs.shape[0]
    x = np.zeros(max(N, 1), dtype=np.float64)
    rep = Report()
    x0a = _c(x0, np.float64) if x0 is not None else None
    lib().orc_pcg27(N, _c(diag, np.float64), _c(off, np.float64), _c(nb26, np.int32), rhs,
                    x0a.ctypes.data if x0a is not None else None, float(tol), int(max_iter), x, C.byref(rep))
    return x[:N], {"iters": rep.iters, "status": rep.status, "rel_res": rep.rel_res}


def hutchinson27(diag, off, nb26, K, seed, tol, max_iter=10000, with_iters=False):
    diag = _c(diag, np.float64)
    N = diag.shape[0]
    s = np.zeros(max(N, 1), dtype=np.float64)
    its = np.zeros(max(K, 1), dtype=np.int32)
    lib().orc_hutchinson27(N, diag, _c(off, np.float64), _c(nb26, np.int32), int(K), C.c_uint64(int(seed)),
                           float(tol), int(max_iter), s, its.ctypes.data)
    if with_iters:
        return s[:N], its[:K]
    return s[:N]


def extract_surface(g: Grid, keys, mu, iso=0.0):
    """Marching-tetrahedra mesh of mu = iso over the band: verts[nv][3], tris[nt][3]."""
    keys = _c(keys, np.uint64)
    mu = _c(mu, np.float64)
    N = keys.shape[0]
    L = lib()
    nv, nt = C.c_int64(), C.c_int64()
    L.orc_extract_surface(C.byref(g), keys, N, mu, float(iso), 0, 0, None, None, C.byref(nv), C.byref(nt))
    verts = np.zeros((max(nv.value, 1), 3), dtype=np.float64)
    tris = np.zeros((max(nt.value, 1), 3), dtype=np.int32)
    L.orc_extract_surface(C.byref(g), keys, N, mu, float(iso), nv.value, nt.value, verts.ctypes.data,
                          tris.ctypes.data, C.byref(nv), C.byref(nt))
    return verts[:nv.value], tris[:nt.value]


def nn_dist2(a, b):
    """Squared distance from each point of a[n][3] to its nearest point of b[m][3]."""
    a = _c(a, np.float64)
    b = _c(b, np.float64)
    d = np.zeros(max(a.shape[0], 1), dtype=np.float64)
    lib().orc_nn_dist2(a, a.shape[0], b, b.shape[0], d)
    return d[:a.shape[0]]


def surface_metrics(pred, gt, thresholds):
    """Eq. (14) and the paper's accuracy, completeness and F-scores from the
    nearest-point distances: CD = mean_p d(p,G)^2 + mean_g d(g,P)^2, accuracy =
    mean_p d(p,G), completeness = mean_g d(g,P), precision/recall = fraction
    within each threshold, F = 2 P R / (P + R).  Sums in ascending index."""
    dp = nn_dist2(pred, gt)
    dg = nn_dist2(gt, pred)
    sp, sg = np.sqrt(dp), np.sqrt(dg)
    acc = {"chamfer": float(np.sum(dp) / len(dp) + np.sum(dg) / len(dg)),
           "accuracy": float(np.sum(sp) / len(sp)), "completeness": float(np.sum(sg) / len(sg)),
           "precision": [], "recall": [], "fscore": []}
    for t in thresholds:
        pr = float(np.count_nonzero(sp < t) / len(sp))
        rc = float(np.count_nonzero(sg < t) / len(sg))
        acc["precision"].append(pr)
        acc["recall"].append(rc)
        acc["fscore"].append(2 * pr * rc / (pr + rc) if pr + rc > 0 else 0.0)
    return acc, dp, dg


def quantize_variance(s):
    s = _c(s, np.float64)
    q = np.zeros(max(s.shape[0], 1), dtype=np.int64)
    lib().orc_quantize_variance(s.shape[0], s, q)
    return q[:s.shape[0]]


def nbv_ray(g: Grid, keys, mu, q, o, d):
    steps = C.c_int64(0)
    sc = lib().orc_nbv_ray(C.byref(g), _c(keys, np.uint64), len(keys), _c(mu, np.float64),
                           _c(q, np.int64), _c(o, np.float64), _c(d, np.float64), C.byref(steps))
    return int(sc), int(steps.value)


def _nbv_all(g: Grid, ray_cam: Cam, keys, mu, q, cands, which, util=None, steps=False):
    """Scores (and plain-walk visit counts) of the listed candidates, candidates in parallel."""
    keys = _c(keys, np.uint64)
    mu = _c(mu, np.float64)
    q = _c(q, np.int64)
    cands = _c(cands, np.float64).reshape(-1, 12)
    if which is not None:
        cands = np.ascontiguousarray(cands[list(which)])
    n = cands.shape[0]
    sc = np.zeros(max(n, 1), dtype=np.int64)
    st = np.zeros(max(n, 1), dtype=np.int64)
    lib().orc_nbv_scores(C.byref(g), C.byref(ray_cam), keys, len(keys), mu, q,
                         C.cast(C.byref(util), C.c_void_p) if util is not None else None, n, cands, sc,
                         st.ctypes.data if steps else None)
    return sc[:n], st[:n]


def nbv_scores(g: Grid, ray_cam: Cam, keys, mu, q, cands, which=None):
    """Summed-variance utility of each listed candidate (eq. 13)."""
    return _nbv_all(g, ray_cam, keys, mu, q, cands, which)[0]


def nbv_scores_steps(g: Grid, ray_cam: Cam, keys, mu, q, cands, which=None):
    """Summed-variance utilities and plain-walk visit counts of the listed candidates."""
    return _nbv_all(g, ray_cam, keys, mu, q, cands, which, steps=True)


def nbv_walk_steps(g: Grid, ray_cam: Cam, keys, mu, q, cands, which=None):
    """Voxels visited by the walks of each listed candidate's rays (as nbv_scores)."""
    return _nbv_all(g, ray_cam, keys, mu, q, cands, which, steps=True)[1]


def nbv_scores_var_reduction(g: Grid, ray_cam: Cam, keys, mu, s, cands, noise=(0.0012, 0.0019, 0.4),
                             which=None):
    """Candidate utilities with the expected-variance-reduction utility."""
    s = _c(s, np.float64)
    u = Utility()
    u.utility = 1
    u.a, u.c, u.z0 = (float(v) for v in noise)
    u.s = s.ctypes.data
    u.smax = float(max(0.0, float(np.max(s)) if len(s) else 0.0))
    q = np.zeros(max(len(s), 1), dtype=np.int64)
    return _nbv_all(g, ray_cam, keys, mu, q, cands, which, util=u)[0]


def pred_depth(g: Grid, cm: Cam, keys, mu, pose):
    """Depth map [H][W] (float32) predicted from the mean for a sensor with camera
    cm at pose [3][4] (camera-z depth of the first band voxel with mu <= 0 on each
    pixel's ray; 0 for none)."""
    keys = _c(keys, np.uint64)
    depth = np.zeros((cm.height, cm.width), dtype=np.float32)
    lib().orc_pred_depth(C.byref(g), C.byref(cm), keys, len(keys), _c(mu, np.float64),
                         _c(pose, np.float64).reshape(12), depth)
    return depth


def nbv_postview(g: Grid, cm: Cam, keys, nbr, deg, Lam, lam, eps, mu, s, pose, K, seed, tol,
                 eps_band=math.inf, noise=(0.0012, 0.0019, 0.4), sigma2_model=0.0, lam_b=0.0, max_iter=10000):
    """Post-view utility of one candidate (Sec. 3.8, eq. 13): the candidate's view is
    predicted from mu, fused as one more view (its Lambda added to the system's,
    then diag(Q') by eq. 11), s' = the Hutchinson estimate on Q' with the same
    probes (eq. 12), and U = sum over |mu| <= eps_band of (s - s') (correctly
    rounded sum).  Returns (U, s', the view's Lambda, the predicted depth, diag')."""
    depth = pred_depth(g, cm, keys, mu, pose)
    dlam, _ = assemble(g, cm, depth[None], np.asarray(pose, dtype=np.float64).reshape(1, 3, 4), keys,
                       noise=noise, sigma2_model=sigma2_model)
    diag_post = precision_diag(np.asarray(Lam, dtype=np.float64) + dlam, deg, lam, eps, lam_b)
    s_post = hutchinson(nbr, diag_post, lam, K, seed, tol, max_iter)
    sel = np.abs(np.asarray(mu)) <= eps_band
    U = math.fsum((np.asarray(s, dtype=np.float64) - s_post)[sel])
    return U, s_post, dlam, depth, diag_post


def nbv_argmax(scores) -> int:
    s = _c(scores, np.int64)
    return int(lib().orc_nbv_argmax(s.shape[0], s))


def features(T, h, tsdf, w, nbr, deg, Lam, acc):
    tsdf = _c(tsdf, np.float64)
    N = tsdf.shape[0]
    out = np.zeros((max(N, 1), 12), dtype=np.float64)
    lib().orc_features(N, int(T), float(h), tsdf, _c(w, np.int32), _c(nbr, np.int32),
                       _c(deg, np.int32), _c(Lam, np.float64), _c(acc, np.float64), out)
    return out[:N]


def full_pipeline(wl, with_acc=False):
    """Band, neighbours, assembly and precision diagonal of a synthetic workload."""
    g = grid_of(wl)
    cm = cam(wl.cam)
    td, wd = tsdf_dense(g, cm, wl.depth, wl.poses)
    keys, bt, bw = band(g, td, wd)
    nbr, deg = neighbours(wl.G, keys)
    res = assemble(g, cm, wl.depth, wl.poses, keys, noise=wl.noise, with_acc=with_acc)
    Lam, b = res[0], res[1]
    diag = precision_diag(Lam, deg, wl.lam, wl.eps, wl.lam_b)
    rhs = anchor_rhs(b, deg, bt, wl.lam_b)
    out = dict(grid=g, cam=cm, tsdf_dense=td, w_dense=wd, keys=keys, tsdf=bt, w=bw, nbr=nbr,
               deg=deg, Lambda=Lam, b=b, diag=diag, rhs=rhs)
    if with_acc:
        out["acc"] = res[2]
    return out
