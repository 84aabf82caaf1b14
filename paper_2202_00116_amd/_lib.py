"""ctypes loader of libdeam.so, the gfx950 HIP library (argument marshalling only).

The library must have been built (``python -m paper_2202_00116_amd.build``);
there is no fallback: importing the ops without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdeam.so")

FAN2D, HELICAL3D = 0, 1
PREC_MIXED, PREC_FP64 = 0, 1
W_AM, W_GRAD, W_VJP, W_STEP_VJP = 0, 1, 2, 3
BP_NONNEG = 1
OP_FORWARD, OP_POLY_MEAN, OP_BACKPROJECT, OP_ITERATE, OP_METAL_TRACE, OP_ITERATE_VJP = 0, 1, 2, 3, 4, 5
OP_PENALTY, OP_ITERATE_PENALIZED, OP_FBP, OP_MAR_INIT = 6, 7, 8, 9

STATUS = {0: "DEAM_OK", -1: "DEAM_ERR_NULL", -2: "DEAM_ERR_SHAPE", -3: "DEAM_ERR_GEOMETRY",
          -4: "DEAM_ERR_WORKSPACE", -5: "DEAM_ERR_HIP", -6: "DEAM_ERR_UNSUPPORTED",
          -7: "DEAM_ERR_VALUE"}

EXPORTS = ("deam_plan_create", "deam_plan_destroy", "deam_plan_sizes", "deam_workspace_size",
           "deam_workspace_size_for",
           "deam_metal_trace", "deam_forward", "deam_poly_mean", "deam_backproject",
           "deam_update", "deam_iterate", "deam_iterate_timed", "deam_iterate_vjp",
           "deam_penalty", "deam_update_penalized", "deam_iterate_penalized",
           "deam_fbp", "deam_nmar", "deam_mar_init", "deam_iterate_os", "deam_dual_workspace_size",
           "deam_iterate_dual", "deam_dilate_mask", "deam_plan_set_bowtie", "deam_pack_mask",
           "deam_iterate_packed", "deam_iterate_sync", "deam_validate_inputs", "deam_poly_mean_noalloc",
           "deam_last_error")


class DeamGeometry(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("n_views", C.c_int32), ("n_rows", C.c_int32), ("n_cols", C.c_int32),
                ("sid", C.c_double), ("sdd", C.c_double), ("dgamma", C.c_double),
                ("col_offset", C.c_double), ("drow_iso", C.c_double), ("beta0", C.c_double),
                ("views_per_rot", C.c_double), ("feed_per_rot", C.c_double)]


class DeamMarParams(C.Structure):
    _fields_ = [("t", C.c_double), ("water", C.c_double * 2), ("air_frac", C.c_double),
                ("bone_frac", C.c_double), ("metal_frac", C.c_double), ("eps", C.c_double)]


class DeamError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libdeam.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2202_00116_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
    G = C.POINTER(DeamGeometry)
    sig = {
        "deam_plan_create": [G, i32, vp, vp, i32, C.POINTER(vp)],
        "deam_plan_destroy": [vp],
        "deam_plan_sizes": [vp, C.POINTER(i64), C.POINTER(i64)],
        "deam_workspace_size": [vp, i32, C.POINTER(sz)],
        "deam_workspace_size_for": [G, i32, i32, C.POINTER(sz)],
        "deam_metal_trace": [vp, vp, dp, vp, vp, vp, sz, vp],
        "deam_forward": [vp, vp, i32, vp, vp, sz, vp],
        "deam_poly_mean": [vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, sz, vp],
        "deam_poly_mean_noalloc": [vp, vp, vp, vp, i32, vp, vp, vp, vp, vp],
        "deam_backproject": [vp, vp, i32, i32, vp, vp, sz, vp],
        "deam_update": [vp, vp, vp, vp, vp, vp],
        "deam_iterate": [vp, vp, vp, vp, vp, vp, i32, vp, vp, sz, vp],
        "deam_iterate_sync": [vp, vp, vp, vp, vp, vp, i32, vp, vp, sz, vp],
        "deam_validate_inputs": [vp, vp, vp, vp, vp, sz, vp],
        "deam_iterate_timed": [vp, vp, vp, vp, vp, vp, i32, vp, vp, sz, vp, vp],
        "deam_iterate_vjp": [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp],
        "deam_penalty": [vp, vp, dp, dp, vp, vp, sz, vp],
        "deam_update_penalized": [vp, vp, vp, vp, vp, vp, dp, dp, vp],
        "deam_iterate_penalized": [vp, vp, vp, vp, vp, dp, dp, i32, vp, vp, sz, vp],
        "deam_fbp": [vp, vp, i32, vp, vp, sz, vp],
        "deam_nmar": [vp, vp, vp, vp, dp, vp, vp],
        "deam_mar_init": [vp, vp, C.POINTER(DeamMarParams), vp, vp, vp, vp, sz, vp],
        "deam_iterate_os": [vp, vp, vp, vp, vp, i32, i32, vp, vp, sz, vp],
        "deam_dual_workspace_size": [vp, vp, C.POINTER(sz)],
        "deam_dilate_mask": [vp, vp, i32, vp, vp],
        "deam_plan_set_bowtie": [vp, vp],
        "deam_pack_mask": [vp, vp, vp, vp],
        "deam_iterate_packed": [vp, vp, vp, vp, vp, i32, vp, vp, sz, vp],
        "deam_iterate_dual": [vp, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp, sz, vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.deam_last_error.argtypes = []
    L.deam_last_error.restype = C.c_char_p
    _lib = L
    return L


def check(rc):
    if rc != 0:
        msg = load().deam_last_error().decode(errors="replace")
        raise DeamError(rc, msg)
    return rc
