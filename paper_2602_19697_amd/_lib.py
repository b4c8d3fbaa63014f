"""ctypes declarations of libbf.so, mirroring include/bf.h one to one."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbf.so")

BF_OK = 0
BF_ERR_INVALID_ARG = 1
BF_ERR_OOM = 2
BF_ERR_CAPACITY = 3
BF_ERR_BREAKDOWN = 4
BF_ERR_NOT_CONVERGED = 5
BF_ERR_HIP = 6
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "CAPACITY", 4: "BREAKDOWN",
                5: "NOT_CONVERGED", 6: "HIP"}

BF_PREC_FP64 = 0
BF_PREC_MIXED = 1
BF_BAND_KEEP_DENSE = 1
BF_UTILITY_SUM_VAR = 0
BF_UTILITY_VAR_REDUCTION = 1
BF_SYSTEM_VOXEL = 0
BF_SYSTEM_TRILINEAR = 1
BF_ORDER_SCENE_MAJOR = 0
BF_ORDER_INTERLEAVED = 1
BF_ORDER_LARGEST_FIRST = 2
BF_MLP_TRAIN = 9282
BF_MLP_PARAMS = 9310


class bf_grid(C.Structure):
    _fields_ = [("G", C.c_int32), ("h", C.c_double), ("origin", C.c_double * 3),
                ("tau", C.c_double), ("band", C.c_double)]


class bf_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double),
                ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class bf_noise(C.Structure):
    _fields_ = [("a", C.c_double), ("c", C.c_double), ("z0", C.c_double),
                ("sigma2_pose_dev", C.c_void_p), ("sigma2_model", C.c_double)]


class bf_prior(C.Structure):
    _fields_ = [("lam", C.c_double), ("eps", C.c_double), ("lambda_b", C.c_double)]


class bf_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32),
                ("use_x0", C.c_int32), ("check_every", C.c_int32)]


class bf_solve_report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("refinements", C.c_int32),
                ("used_warm_start", C.c_int32), ("rel_res", C.c_double), ("seconds", C.c_double),
                ("col_iters", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class bf_probe_opts(C.Structure):
    _fields_ = [("K", C.c_int32), ("precision", C.c_int32), ("seed", C.c_uint64),
                ("tol", C.c_double), ("max_iter", C.c_int32)]


class bf_schedule(C.Structure):
    _fields_ = [("rows_per_tile", C.c_int32), ("blocks_per_cu", C.c_int32), ("order", C.c_int32),
                ("xcd_aware", C.c_int32), ("persistent", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class bf_band_arrays(C.Structure):
    _fields_ = [("n", C.c_int64), ("dense_side", C.c_int32), ("keys", C.c_void_p),
                ("tsdf", C.c_void_p), ("w", C.c_void_p), ("nbr", C.c_void_p), ("deg", C.c_void_p),
                ("dense_tsdf", C.c_void_p), ("dense_w", C.c_void_p), ("tsdf_voxel_views", C.c_int64),
                ("tsdf_box_tests", C.c_int64), ("tsdf_tile_tests", C.c_int64)]


class bf_system_arrays(C.Structure):
    _fields_ = [("n", C.c_int64), ("Lambda", C.c_void_p), ("b", C.c_void_p), ("rhs", C.c_void_p),
                ("diag", C.c_void_p), ("diag32", C.c_void_p), ("acc", C.c_void_p), ("kind", C.c_int32),
                ("off", C.c_void_p), ("nb26", C.c_void_p), ("n_samples", C.c_int64), ("n_cells", C.c_int64)]


class bf_mesh_arrays(C.Structure):
    _fields_ = [("n_vert", C.c_int64), ("n_tri", C.c_int64), ("verts", C.c_void_p), ("tris", C.c_void_p)]


class bf_metrics(C.Structure):
    _fields_ = [("n_pred", C.c_int64), ("n_gt", C.c_int64), ("chamfer", C.c_double), ("accuracy", C.c_double),
                ("completeness", C.c_double), ("n_thr", C.c_int32), ("thr", C.c_double * 8),
                ("precision", C.c_double * 8), ("recall", C.c_double * 8), ("fscore", C.c_double * 8)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class bf_allocator(C.Structure):
    _fields_ = [("user", C.c_void_p), ("alloc", ALLOC_FN), ("release", RELEASE_FN)]


class bf_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double)]


P = C.c_void_p
PP = C.POINTER(C.c_void_p)

# name: (restype, argtypes)
SIGNATURES = {
    "bf_version": (C.c_char_p, []),
    "bf_create": (C.c_int, [PP, C.c_int32, P, C.POINTER(bf_allocator)]),
    "bf_destroy": (C.c_int, [P]),
    "bf_set_stream": (C.c_int, [P, P]),
    "bf_last_error": (C.c_char_p, [P]),
    "bf_build_band": (C.c_int, [P, C.POINTER(bf_grid), C.POINTER(bf_camera), C.c_int32, P, P,
                                C.c_uint32, PP, C.POINTER(C.c_int64)]),
    "bf_band_view": (C.c_int, [P, C.POINTER(bf_band_arrays)]),
    "bf_band_free": (C.c_int, [P, P]),
    "bf_assemble": (C.c_int, [P, P, C.POINTER(bf_camera), C.c_int32, P, P, C.POINTER(bf_noise),
                              C.POINTER(bf_prior), PP]),
    "bf_assemble_trilinear": (C.c_int, [P, P, C.POINTER(bf_camera), C.c_int32, P, P, C.POINTER(bf_noise),
                                        C.POINTER(bf_prior), C.c_int32, PP, C.POINTER(C.c_int64)]),
    "bf_assemble_more": (C.c_int, [P, P, C.POINTER(bf_camera), C.c_int32, P, P, C.POINTER(bf_noise), PP]),
    "bf_system_view": (C.c_int, [P, C.POINTER(bf_system_arrays)]),
    "bf_system_assembly_views": (C.c_int, [P, P, C.POINTER(C.c_int64)]),
    "bf_extract_surface": (C.c_int, [P, P, P, C.c_double, PP, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "bf_mesh_view": (C.c_int, [P, C.POINTER(bf_mesh_arrays)]),
    "bf_mesh_free": (C.c_int, [P, P]),
    "bf_surface_metrics": (C.c_int, [P, P, C.c_int64, P, C.c_int64, C.c_int32, C.POINTER(C.c_double),
                                     C.POINTER(bf_metrics), P, P]),
    "bf_system_free": (C.c_int, [P, P]),
    "bf_apply_Q": (C.c_int, [P, P, P, P]),
    "bf_features": (C.c_int, [P, P, P]),
    "bf_pcg_solve": (C.c_int, [P, P, C.POINTER(bf_solve_opts), P, P, C.POINTER(bf_solve_report)]),
    "bf_pcg_solve_noalloc": (C.c_int, [P, P, C.POINTER(bf_solve_opts), P, P, C.POINTER(bf_solve_report)]),
    "bf_pcg_noalloc_max_n": (C.c_int64, [C.c_int32]),
    "bf_diag_estimate": (C.c_int, [P, P, C.POINTER(bf_probe_opts), P, P,
                                   C.POINTER(bf_solve_report)]),
    "bf_nbv_score": (C.c_int, [P, P, P, P, C.c_int32, P, C.POINTER(bf_camera), C.c_int32,
                               C.POINTER(bf_noise), P, C.POINTER(C.c_int32)]),
    "bf_nbv_walk_steps": (C.c_int, [P, C.POINTER(C.c_int64)]),
    "bf_predict_depth": (C.c_int, [P, P, P, P, C.POINTER(bf_camera), P]),
    "bf_nbv_postview": (C.c_int, [P, P, P, P, C.c_int32, P, C.c_int32, P, C.POINTER(bf_camera), C.POINTER(bf_noise),
                                  C.POINTER(bf_probe_opts), C.c_double, C.c_int32, P, C.POINTER(C.c_int32), P, P]),
    "bf_diag_estimate_batched": (C.c_int, [P, P, C.c_int32, C.POINTER(bf_probe_opts), C.POINTER(bf_schedule),
                                           P, C.POINTER(bf_solve_report)]),
    "bf_pcg_solve_batched": (C.c_int, [P, P, C.c_int32, C.POINTER(bf_solve_opts), C.POINTER(bf_schedule), P,
                                       C.POINTER(bf_solve_report)]),
    "bf_autotune_batch": (C.c_int, [P, P, C.c_int32, C.POINTER(bf_probe_opts), P, C.POINTER(bf_schedule),
                                    C.c_char_p, C.c_size_t]),
    "bf_mlp_forward": (C.c_int, [P, P, P, C.c_int64, P]),
    "bf_warm_start": (C.c_int, [P, P, P, P, P, P]),
    "bf_warm_start_targets": (C.c_int, [P, P, P, P, C.c_double, C.c_double, P]),
    "bf_mlp_grad": (C.c_int, [P, P, P, P, C.c_int64, P, C.c_int64, P, P]),
    "bf_adam_step": (C.c_int, [P, P, P, P, P, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float]),
    "bf_set_timing": (C.c_int, [P, C.c_int32]),
    "bf_get_timings": (C.c_int, [P, C.POINTER(bf_kernel_time), C.c_int32, C.POINTER(C.c_int32)]),
}

_lib = None


def load():
    """Load libbf.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the gfx950 HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L
