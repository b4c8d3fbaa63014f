"""Python binding of the gfx950 BayesFusion-SDF library (libbf.so).

Argument marshalling only: torch supplies device memory and the stream, every
step of the method runs in the library's HIP kernels.  Function names follow
the C ABI in include/bf.h (bf_build_band, bf_assemble, bf_pcg_solve,
bf_diag_estimate, bf_nbv_score, ...).  Importing this package does not load
the library; the first Context does, and fails loudly if it is not built.
"""
from __future__ import annotations

import ctypes as C
import math
import dataclasses

import torch

from . import _lib as L

__all__ = ["Context", "Band", "System", "BFError", "L"]


class BFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr()


class _DevArray:
    """Minimal __cuda_array_interface__ view of library-owned device memory."""

    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"data": (int(ptr), False), "shape": tuple(shape),
                                         "typestr": typestr, "version": 2, "strides": None}


_TYPESTR = {torch.float64: "<f8", torch.float32: "<f4", torch.int32: "<i4", torch.int64: "<i8",
            torch.uint64: "<u8"}


_hip = None


def _hip_memcpy_d2d(dst: int, src: int, nbytes: int, stream) -> None:
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        _hip.hipMemcpyAsync.restype = C.c_int
    st = _hip.hipMemcpyAsync(C.c_void_p(dst), C.c_void_p(src), C.c_size_t(nbytes), 3,
                             C.c_void_p(stream.cuda_stream))
    if st != 0:
        raise RuntimeError(f"hipMemcpyAsync failed ({st})")


def _view(ptr, shape, dtype, device, copy=False):
    """Tensor over library-owned device memory (aliasing), or a stream-ordered copy."""
    if not ptr or any(s == 0 for s in shape):
        return torch.empty(shape, dtype=dtype, device=device)
    if not copy:
        try:
            return torch.as_tensor(_DevArray(ptr, shape, _TYPESTR[dtype]), device=device)
        except Exception:
            pass
    out = torch.empty(shape, dtype=dtype, device=device)
    _hip_memcpy_d2d(out.data_ptr(), ptr, out.numel() * out.element_size(),
                    torch.cuda.current_stream(device))
    return out


def grid_struct(G, h, origin, tau, band) -> L.bf_grid:
    g = L.bf_grid()
    g.G, g.h, g.tau, g.band = int(G), float(h), float(tau), float(band)
    for a in range(3):
        g.origin[a] = float(origin[a])
    return g


def camera_struct(cam) -> L.bf_camera:
    c = L.bf_camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    return c


def noise_struct(a=0.0012, c=0.0019, z0=0.4, sigma2_pose=None, sigma2_model=0.0) -> L.bf_noise:
    n = L.bf_noise()
    n.a, n.c, n.z0, n.sigma2_model = float(a), float(c), float(z0), float(sigma2_model)
    n.sigma2_pose_dev = _ptr(sigma2_pose)
    return n


@dataclasses.dataclass
class Mesh:
    ctx: "Context"
    handle: C.c_void_p
    n_vert: int
    n_tri: int

    def arrays(self) -> dict:
        a = L.bf_mesh_arrays()
        self.ctx._check(self.ctx.lib.bf_mesh_view(self.handle, C.byref(a)))
        dev = self.ctx.device
        return {"verts": _view(a.verts, (int(a.n_vert), 3), torch.float64, dev),
                "tris": _view(a.tris, (int(a.n_tri), 3), torch.int32, dev)}

    def free(self):
        if self.handle:
            self.ctx.lib.bf_mesh_free(self.ctx.handle, self.handle)
            self.handle = None


@dataclasses.dataclass
class Band:
    ctx: "Context"
    handle: C.c_void_p
    n: int

    def info(self) -> dict:
        """The band's scalar fields only (no tensor views)."""
        a = L.bf_band_arrays()
        self.ctx._check(self.ctx.lib.bf_band_view(self.handle, C.byref(a)))
        return {"n": int(a.n), "dense_side": int(a.dense_side), "tsdf_voxel_views": int(a.tsdf_voxel_views),
                "tsdf_box_tests": int(a.tsdf_box_tests), "tsdf_tile_tests": int(a.tsdf_tile_tests)}

    def arrays(self) -> dict:
        a = L.bf_band_arrays()
        self.ctx._check(self.ctx.lib.bf_band_view(self.handle, C.byref(a)))
        dev, n = self.ctx.device, int(a.n)
        out = {"keys": _view(a.keys, (n,), torch.uint64, dev),
               "tsdf": _view(a.tsdf, (n,), torch.float64, dev),
               "w": _view(a.w, (n,), torch.int32, dev),
               "nbr": _view(a.nbr, (n, 6), torch.int32, dev),
               "deg": _view(a.deg, (n,), torch.int32, dev),
               "dense_side": int(a.dense_side), "tsdf_voxel_views": int(a.tsdf_voxel_views),
               "tsdf_box_tests": int(a.tsdf_box_tests), "tsdf_tile_tests": int(a.tsdf_tile_tests)}
        P3 = int(a.dense_side) ** 3
        if a.dense_tsdf:
            out["dense_tsdf"] = _view(a.dense_tsdf, (P3,), torch.float64, dev)
            out["dense_w"] = _view(a.dense_w, (P3,), torch.int32, dev)
        return out

    def free(self):
        if self.handle:
            self.ctx.lib.bf_band_free(self.ctx.handle, self.handle)
            self.handle = None


@dataclasses.dataclass
class System:
    ctx: "Context"
    handle: C.c_void_p
    n: int
    band: Band

    def arrays(self) -> dict:
        a = L.bf_system_arrays()
        self.ctx._check(self.ctx.lib.bf_system_view(self.handle, C.byref(a)))
        dev, n = self.ctx.device, int(a.n)
        out = {"Lambda": _view(a.Lambda, (n,), torch.float64, dev),
               "b": _view(a.b, (n,), torch.float64, dev),
               "rhs": _view(a.rhs, (n,), torch.float64, dev),
               "diag": _view(a.diag, (n,), torch.float64, dev),
               "diag32": _view(a.diag32, (n,), torch.float32, dev),
               "kind": int(a.kind), "n_samples": int(a.n_samples), "n_cells": int(a.n_cells)}
        if a.kind == L.BF_SYSTEM_VOXEL:
            out["acc"] = _view(a.acc, (n, 5), torch.float64, dev)
        else:
            # stored slot-major [26][N]; shown as [N][26] (a transposed view)
            out["off"] = _view(a.off, (26, n), torch.float64, dev).t()
            out["nb26"] = _view(a.nb26, (26, n), torch.int32, dev).t()
        return out

    def assembly_views(self) -> int:
        """(band voxel, view) pairs the assembly went through (synchronises)."""
        out = C.c_int64(0)
        self.ctx._check(self.ctx.lib.bf_system_assembly_views(self.ctx.handle, self.handle, C.byref(out)))
        return int(out.value)

    def free(self):
        if self.handle:
            self.ctx.lib.bf_system_free(self.ctx.handle, self.handle)
            self.handle = None


def _torch_allocator(idx):
    """A bf_allocator that hands out torch's caching-allocator memory on device
    idx (blocks are cached by torch and reused on the context's stream)."""
    def alloc(user, nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=idx, stream=int(stream or 0))
        except Exception:  # torch raises on out-of-memory: the library reports BF_ERR_OOM
            return None

    def release(user, ptr, stream):
        torch.cuda.caching_allocator_delete(int(ptr))

    a = L.bf_allocator()
    a.user = None
    a.alloc = L.ALLOC_FN(alloc)
    a.release = L.RELEASE_FN(release)
    return a


class Context:
    """One bf_ctx on a torch CUDA (HIP) device, ordered on torch's current stream.

    allocator="torch" (default) gives the memory of bands, systems and meshes
    from torch's caching allocator (through the C ABI's bf_allocator hook);
    allocator=None leaves it to the library's own stream-ordered pool."""

    def __init__(self, device="cuda:0", stream=None, allocator="torch"):
        self.lib = L.load()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the library runs on a GPU device")
        idx = self.device.index if self.device.index is not None else torch.cuda.current_device()
        self.device = torch.device("cuda", idx)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        if isinstance(allocator, L.bf_allocator):
            self._alloc = allocator  # a caller's own provider (kept alive with the context)
        elif allocator == "torch":
            self._alloc = _torch_allocator(idx)
        elif allocator is None:
            self._alloc = None
        else:
            raise ValueError("allocator must be 'torch', None or a bf_allocator")
        h = C.c_void_p()
        st = self.lib.bf_create(C.byref(h), idx, C.c_void_p(s.cuda_stream),
                                C.byref(self._alloc) if self._alloc is not None else None)
        if st != 0:
            raise BFError(st, "bf_create failed")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.bf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow=()):
        if st != 0 and st not in allow:
            raise BFError(st, self.lib.bf_last_error(self.handle).decode())
        return st

    # ---------------------------------------------------------- instrumentation
    def bf_set_timing(self, enable: bool):
        self._check(self.lib.bf_set_timing(self.handle, 1 if enable else 0))

    def bf_get_timings(self) -> dict:
        """{kernel name: (launches, total ms)} since the last call (synchronises)."""
        cap = 64
        arr = (L.bf_kernel_time * cap)()
        n = C.c_int32()
        self._check(self.lib.bf_get_timings(self.handle, arr, cap, C.byref(n)))
        return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n.value)}

    # ---------------------------------------------------------- band
    def bf_build_band(self, grid: L.bf_grid, cam, depth, poses, keep_dense=False) -> Band:
        T = int(depth.shape[0]) if depth is not None else 0
        h = C.c_void_p()
        n = C.c_int64()
        self._check(self.lib.bf_build_band(self.handle, C.byref(grid), C.byref(camera_struct(cam)), T,
                                           _ptr(depth), _ptr(poses),
                                           L.BF_BAND_KEEP_DENSE if keep_dense else 0, C.byref(h),
                                           C.byref(n)))
        return Band(self, h, int(n.value))

    # ---------------------------------------------------------- system
    def bf_assemble(self, band: Band, cam, depth, poses, noise: L.bf_noise, lam, eps,
                    lam_b=0.0) -> System:
        pr = L.bf_prior()
        pr.lam, pr.eps, pr.lambda_b = float(lam), float(eps), float(lam_b)
        h = C.c_void_p()
        self._check(self.lib.bf_assemble(self.handle, band.handle, C.byref(camera_struct(cam)),
                                         int(depth.shape[0]), _ptr(depth), _ptr(poses), C.byref(noise),
                                         C.byref(pr), C.byref(h)))
        return System(self, h, band.n, band)

    def bf_assemble_more(self, sys: System, cam, depth, poses, noise: L.bf_noise) -> System:
        """sys with the views depth [T][H][W] / poses [T][3][4] appended (a new system)."""
        h = C.c_void_p()
        self._check(self.lib.bf_assemble_more(self.handle, sys.handle, C.byref(camera_struct(cam)),
                                              int(depth.shape[0]), _ptr(depth), _ptr(poses), C.byref(noise),
                                              C.byref(h)))
        return System(self, h, sys.n, sys.band)

    def bf_assemble_trilinear(self, band: Band, cam, depth, poses, noise: L.bf_noise, lam, eps, lam_b=0.0,
                              samples_per_side=4) -> System:
        """Trilinear pixel-centric rows (eq. 4): 2S+1 samples per pixel, 27-point Q."""
        pr = L.bf_prior()
        pr.lam, pr.eps, pr.lambda_b = float(lam), float(eps), float(lam_b)
        h = C.c_void_p()
        ns = C.c_int64()
        self._check(self.lib.bf_assemble_trilinear(self.handle, band.handle, C.byref(camera_struct(cam)),
                                                   int(depth.shape[0]), _ptr(depth), _ptr(poses), C.byref(noise),
                                                   C.byref(pr), int(samples_per_side), C.byref(h), C.byref(ns)))
        return System(self, h, band.n, band)

    # ---------------------------------------------------------- surface
    def bf_extract_surface(self, band: Band, mu, iso=0.0) -> Mesh:
        """Marching-tetrahedra iso-surface mu = iso over the band (Algorithm 1 step 7)."""
        h = C.c_void_p()
        nv, nt = C.c_int64(), C.c_int64()
        self._check(self.lib.bf_extract_surface(self.handle, band.handle, _ptr(mu), float(iso), C.byref(h),
                                                C.byref(nv), C.byref(nt)))
        return Mesh(self, h, int(nv.value), int(nt.value))

    def bf_surface_metrics(self, pred, gt, thresholds=(), with_distances=False):
        """Chamfer (eq. 14), accuracy, completeness and F-scores between point sets."""
        thr = (C.c_double * max(len(thresholds), 1))(*[float(t) for t in thresholds])
        m = L.bf_metrics()
        dp = torch.empty(pred.shape[0], dtype=torch.float64, device=self.device) if with_distances else None
        dg = torch.empty(gt.shape[0], dtype=torch.float64, device=self.device) if with_distances else None
        self._check(self.lib.bf_surface_metrics(self.handle, _ptr(pred), int(pred.shape[0]), _ptr(gt),
                                                int(gt.shape[0]), len(thresholds), thr, C.byref(m), _ptr(dp),
                                                _ptr(dg)))
        k = int(m.n_thr)
        out = {"chamfer": m.chamfer, "accuracy": m.accuracy, "completeness": m.completeness,
               "thresholds": list(m.thr[:k]), "precision": list(m.precision[:k]), "recall": list(m.recall[:k]),
               "fscore": list(m.fscore[:k])}
        if with_distances:
            out["d_pred"], out["d_gt"] = dp, dg
        return out

    def bf_apply_Q(self, sys: System, p):
        q = torch.empty_like(p)
        self._check(self.lib.bf_apply_Q(self.handle, sys.handle, _ptr(p), _ptr(q)))
        return q

    def bf_features(self, sys: System):
        f = torch.empty((sys.n, 12), dtype=torch.float32, device=self.device)
        self._check(self.lib.bf_features(self.handle, sys.handle, _ptr(f)))
        return f

    # ---------------------------------------------------------- batched solves
    @staticmethod
    def schedule(rows_per_tile=256, blocks_per_cu=0, order=L.BF_ORDER_SCENE_MAJOR, xcd_aware=1, persistent=1):
        s = L.bf_schedule()
        s.rows_per_tile, s.blocks_per_cu, s.order, s.xcd_aware = rows_per_tile, blocks_per_cu, order, xcd_aware
        s.persistent = persistent
        return s

    def _batch_args(self, systems, outs):
        n = len(systems)
        sys_arr = (C.c_void_p * n)(*[s.handle.value if isinstance(s.handle, C.c_void_p) else s.handle
                                     for s in systems])
        out_arr = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        reps = (L.bf_solve_report * n)()
        return n, sys_arr, out_arr, reps

    def bf_diag_estimate_batched(self, systems, K, seed, tol, max_iter=10000, precision=L.BF_PREC_MIXED,
                                 schedule=None, allow_fail=False):
        o = L.bf_probe_opts()
        o.K, o.precision, o.seed, o.tol, o.max_iter = int(K), int(precision), int(seed), float(tol), int(max_iter)
        outs = [torch.empty(s.n, dtype=torch.float64, device=self.device) for s in systems]
        n, sa, oa, reps = self._batch_args(systems, outs)
        st = self.lib.bf_diag_estimate_batched(self.handle, sa, n, C.byref(o),
                                               C.byref(schedule) if schedule is not None else None, oa, reps)
        self._check(st, allow=(L.BF_ERR_NOT_CONVERGED, L.BF_ERR_BREAKDOWN) if allow_fail else ())
        return outs, [r.as_dict() for r in reps]

    def bf_pcg_solve_batched(self, systems, tol, max_iter=10000, precision=L.BF_PREC_MIXED, schedule=None,
                             allow_fail=False):
        o = L.bf_solve_opts()
        o.tol, o.max_iter, o.precision, o.use_x0, o.check_every = float(tol), int(max_iter), int(precision), 0, 0
        outs = [torch.empty(s.n, dtype=torch.float64, device=self.device) for s in systems]
        n, sa, oa, reps = self._batch_args(systems, outs)
        st = self.lib.bf_pcg_solve_batched(self.handle, sa, n, C.byref(o),
                                           C.byref(schedule) if schedule is not None else None, oa, reps)
        self._check(st, allow=(L.BF_ERR_NOT_CONVERGED, L.BF_ERR_BREAKDOWN) if allow_fail else ())
        return outs, [r.as_dict() for r in reps]

    def bf_autotune_batch(self, systems, K, seed, tol, max_iter=10000, precision=L.BF_PREC_MIXED):
        import json as _json
        o = L.bf_probe_opts()
        o.K, o.precision, o.seed, o.tol, o.max_iter = int(K), int(precision), int(seed), float(tol), int(max_iter)
        outs = [torch.empty(s.n, dtype=torch.float64, device=self.device) for s in systems]
        n, sa, oa, _ = self._batch_args(systems, outs)
        best = L.bf_schedule()
        buf = C.create_string_buffer(1 << 16)
        self._check(self.lib.bf_autotune_batch(self.handle, sa, n, C.byref(o), oa, C.byref(best), buf, len(buf)))
        return best, _json.loads(buf.value.decode())

    # ---------------------------------------------------------- learned warm start
    def bf_mlp_forward(self, params, feat):
        out = torch.empty((feat.shape[0], 2), dtype=torch.float32, device=self.device)
        self._check(self.lib.bf_mlp_forward(self.handle, _ptr(params), _ptr(feat), int(feat.shape[0]), _ptr(out)))
        return out

    def bf_warm_start(self, sys: System, params, feat=None, mean=True, logvar=True):
        """x0 and log-variance starts; feat None computes the features in the same pass."""
        x0 = torch.empty(sys.n, dtype=torch.float64, device=self.device) if mean else None
        lv = torch.empty(sys.n, dtype=torch.float32, device=self.device) if logvar else None
        self._check(self.lib.bf_warm_start(self.handle, sys.handle, _ptr(params), _ptr(feat), _ptr(x0), _ptr(lv)))
        return x0, lv

    def bf_warm_start_targets(self, sys: System, mu, s, clamp_lo=1e-3, clamp_hi=1e3, out=None):
        tgt = out if out is not None else torch.empty((sys.n, 2), dtype=torch.float32, device=self.device)
        self._check(self.lib.bf_warm_start_targets(self.handle, sys.handle, _ptr(mu), _ptr(s), float(clamp_lo),
                                                   float(clamp_hi), _ptr(tgt)))
        return tgt

    def bf_mlp_grad(self, params, feat, target, idx, grad=None, loss=None):
        grad = grad if grad is not None else torch.empty(L.BF_MLP_TRAIN, dtype=torch.float32, device=self.device)
        loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=self.device)
        self._check(self.lib.bf_mlp_grad(self.handle, _ptr(params), _ptr(feat), _ptr(target), int(feat.shape[0]),
                                         _ptr(idx), int(idx.shape[0]), _ptr(grad), _ptr(loss)))
        return grad, loss

    def bf_adam_step(self, params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.lib.bf_adam_step(self.handle, _ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(step),
                                          float(lr), float(beta1), float(beta2), float(eps)))

    # ---------------------------------------------------------- solves
    def _pcg(self, fn, sys, tol, max_iter, precision, x0, rhs, check_every, out, allow_fail):
        o = L.bf_solve_opts()
        o.tol, o.max_iter, o.precision = float(tol), int(max_iter), int(precision)
        o.use_x0 = 1 if x0 is not None else 0
        o.check_every = int(check_every)
        x = out if out is not None else torch.empty(sys.n, dtype=torch.float64, device=self.device)
        if x0 is not None and x0.data_ptr() != x.data_ptr():
            x.copy_(x0)
        rep = L.bf_solve_report()
        st = fn(self.handle, sys.handle, C.byref(o), _ptr(rhs), _ptr(x), C.byref(rep))
        self._check(st, allow=(L.BF_ERR_NOT_CONVERGED, L.BF_ERR_BREAKDOWN) if allow_fail else ())
        return x, rep.as_dict()

    def bf_pcg_solve(self, sys: System, tol, max_iter=10000, precision=L.BF_PREC_FP64, x0=None,
                     rhs=None, check_every=0, out=None, allow_fail=False):
        return self._pcg(self.lib.bf_pcg_solve, sys, tol, max_iter, precision, x0, rhs, check_every, out,
                         allow_fail)

    def bf_pcg_solve_noalloc(self, sys: System, tol, max_iter=10000, precision=L.BF_PREC_FP64, x0=None,
                             rhs=None, check_every=0, out=None, allow_fail=False):
        """bf_pcg_solve with the library's static per-GPU scratch (no allocation
        inside the call); pass `out` (and `x0` in it) to allocate nothing here either."""
        return self._pcg(self.lib.bf_pcg_solve_noalloc, sys, tol, max_iter, precision, x0, rhs, check_every, out,
                         allow_fail)

    def bf_pcg_noalloc_max_n(self, precision=L.BF_PREC_FP64) -> int:
        return int(self.lib.bf_pcg_noalloc_max_n(int(precision)))

    def bf_diag_estimate(self, sys: System, K, seed, tol, max_iter=10000, precision=L.BF_PREC_FP64,
                         logvar=None, out=None, allow_fail=False):
        o = L.bf_probe_opts()
        o.K, o.precision, o.seed, o.tol, o.max_iter = int(K), int(precision), int(seed), float(tol), int(max_iter)
        s = out if out is not None else torch.empty(sys.n, dtype=torch.float64, device=self.device)
        rep = L.bf_solve_report()
        st = self.lib.bf_diag_estimate(self.handle, sys.handle, C.byref(o), _ptr(logvar), _ptr(s), C.byref(rep))
        self._check(st, allow=(L.BF_ERR_NOT_CONVERGED, L.BF_ERR_BREAKDOWN) if allow_fail else ())
        return s, rep.as_dict()

    # ---------------------------------------------------------- NBV
    def bf_nbv_walk_steps(self) -> int:
        v = C.c_int64()
        self._check(self.lib.bf_nbv_walk_steps(self.handle, C.byref(v)))
        return int(v.value)

    def bf_predict_depth(self, band: Band, mu, pose, cam):
        """Depth map [H][W] (float32) a sensor with camera cam would see from pose [3][4]."""
        c = camera_struct(cam)
        depth = torch.empty((c.height, c.width), dtype=torch.float32, device=self.device)
        self._check(self.lib.bf_predict_depth(self.handle, band.handle, _ptr(mu), _ptr(pose), C.byref(c),
                                              _ptr(depth)))
        return depth

    def bf_nbv_postview(self, sys: System, mu, s, cands, which, cam, noise: L.bf_noise, K, seed, tol,
                        precision=L.BF_PREC_MIXED, eps_band=None, warm=True, max_iter=10000, keep_s=False):
        """Post-view utilities U = sum_{|mu| <= eps_band} (s - s') of the candidates `which`
        (eq. 13); eps_band None takes every band voxel.  Returns (utilities, best
        candidate index, s' [len(which)][N] or None, reports)."""
        which = [int(i) for i in which]
        n_sel = len(which)
        idx = (C.c_int32 * max(n_sel, 1))(*which)
        util = (C.c_double * max(n_sel, 1))()
        reps = (L.bf_solve_report * max(n_sel, 1))()
        best = C.c_int32(-1)
        o = L.bf_probe_opts()
        o.K, o.precision, o.seed, o.tol, o.max_iter = int(K), int(precision), int(seed), float(tol), int(max_iter)
        s_post = torch.empty((n_sel, sys.n), dtype=torch.float64, device=self.device) if keep_s else None
        eps = math.inf if eps_band is None else float(eps_band)
        self._check(self.lib.bf_nbv_postview(self.handle, sys.handle, _ptr(mu), _ptr(s), int(cands.shape[0]),
                                             _ptr(cands), n_sel, idx, C.byref(camera_struct(cam)), C.byref(noise),
                                             C.byref(o), eps, 1 if warm else 0, util, C.byref(best),
                                             _ptr(s_post), reps))
        return [util[i] for i in range(n_sel)], int(best.value), s_post, [reps[i].as_dict() for i in range(n_sel)]

    def bf_nbv_score(self, band: Band, mu, s, cands, ray_cam, utility=L.BF_UTILITY_SUM_VAR, noise=None):
        n = int(cands.shape[0])
        scores = torch.empty(n, dtype=torch.int64, device=self.device)
        best = C.c_int32(-1)
        self._check(self.lib.bf_nbv_score(self.handle, band.handle, _ptr(mu), _ptr(s), n, _ptr(cands),
                                          C.byref(camera_struct(ray_cam)), int(utility),
                                          C.byref(noise) if noise is not None else None,
                                          _ptr(scores), C.byref(best)))
        return scores, int(best.value)
