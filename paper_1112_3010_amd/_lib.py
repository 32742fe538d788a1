"""ctypes view of libdt.so (the C ABI declared in include/dt.h).

Only argument marshalling lives here.  The library is loaded from this
package's directory; if it is missing the import fails loudly (there is no
CPU fallback).
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdt.so")

DT_OK, DT_E_ARG, DT_E_RANGE, DT_E_PRECISION, DT_E_WORKSPACE, DT_E_HIP, DT_E_UNSUPPORTED = range(7)
DT_FP32_SCALED, DT_FP64, DT_AUTO, DT_FP64X2, DT_FP64X4 = 0, 1, 2, 3, 4
DT_OUT_S, DT_OUT_GRAD, DT_OUT_HESS, DT_OUT_SIGN, DT_OUT_BACKWARD, DT_OUT_CURV = 1, 2, 4, 8, 16, 32
DT_SHAPE_POLYGON, DT_SHAPE_MESH = 1, 2
DT_STATIC_WORKSPACE_BYTES = 64 << 20

EXPORTED = (
    "dt_create_plan", "dt_create_plan_reduced", "dt_plan_workspace_size", "dt_plan_set_workspace", "dt_plan_set_static_workspace",
    "dt_plan_info", "dt_destroy_plan",
    "dt_distance", "dt_gradient", "dt_hessian", "dt_sign", "dt_forward", "dt_backward",
    "dt_last_error", "dt_last_stats", "dt_plan_set_timing", "dt_plan_timings", "dt_plan_reset_timings",
    "dt_create_batch_plan", "dt_batch_workspace_size", "dt_batch_set_workspace", "dt_batch_instance_info",
    "dt_batch_set_tiles", "dt_batch_get_tiles", "dt_batch_set_schedule", "dt_batch_get_schedule",
    "dt_batch_set_graph", "dt_forward_batched", "dt_batch_autotune",
    "dt_batch_last_error", "dt_batch_stats", "dt_destroy_batch_plan",
    "dt_status_str",
)


class DtShape(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("points", ctypes.c_void_p),
        ("n_points", ctypes.c_int64),
        ("vertices", ctypes.c_void_p),
        ("n_vertices", ctypes.c_int64),
        ("faces", ctypes.c_void_p),
        ("n_faces", ctypes.c_int64),
    ]


class DtOutputs(ctypes.Structure):
    _fields_ = [
        ("S", ctypes.c_void_p),
        ("grad", ctypes.c_void_p),
        ("hess", ctypes.c_void_p),
        ("label", ctypes.c_void_p),
        ("mu", ctypes.c_void_p),
        ("signed_outputs", ctypes.c_int),
        ("curv", ctypes.c_void_p),
    ]


class DtPlanInfo(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("dims", ctypes.c_int64 * 3),
        ("padded", ctypes.c_int64 * 3),
        ("spacing", ctypes.c_double * 3),
        ("origin", ctypes.c_double * 3),
        ("tau", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("out_mask", ctypes.c_uint),
        ("c_theta", ctypes.c_double),
        ("kernel_l1", ctypes.c_double),
        ("unit_roundoff", ctypes.c_double),
        ("workspace_bytes", ctypes.c_size_t),
        ("n_tables", ctypes.c_int),
        ("k_max", ctypes.c_int64),
        ("cut", ctypes.c_int * 3),
    ]


class DtCallStats(ctypes.Structure):
    _fields_ = [
        ("g_l2", ctypes.c_double),
        ("theta", ctypes.c_double),
        ("s_max", ctypes.c_double),
        ("dL_dtau", ctypes.c_double),
        ("error_bits", ctypes.c_uint32),
    ]


class DtPassTiming(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class DtInstanceDesc(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int64 * 2),
        ("spacing", ctypes.c_double * 2),
        ("origin", ctypes.c_double * 2),
        ("tau", ctypes.c_double),
        ("k_max", ctypes.c_int64),
    ]


class DtBatchInstanceInfo(ctypes.Structure):
    _fields_ = [
        ("padded", ctypes.c_int64 * 2),
        ("node_offset", ctypes.c_int64),
        ("total_nodes", ctypes.c_int64),
        ("precision", ctypes.c_int),
        ("kernel_l1", ctypes.c_double),
    ]


class DtBatchTiles(ctypes.Structure):
    _fields_ = [("col_nb", ctypes.c_int), ("col_threads", ctypes.c_int), ("row_threads", ctypes.c_int)]


class DtError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} (status {status})")


_lib = None


def load():
    """Load libdt.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1112_3010_amd.build` "
                          "(the distance-field path has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.dt_create_plan.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(i64), ctypes.POINTER(dbl),
                                   ctypes.POINTER(dbl), dbl, ctypes.c_int, ctypes.c_uint, dbl, i64, dbl]
    lib.dt_create_plan_reduced.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(i64),
                                           ctypes.POINTER(dbl), ctypes.POINTER(dbl), dbl, ctypes.c_int, ctypes.c_uint,
                                           i64, dbl]
    lib.dt_plan_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.dt_plan_set_workspace.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.dt_plan_set_static_workspace.argtypes = [vp, vp]
    lib.dt_plan_info.argtypes = [vp, ctypes.POINTER(DtPlanInfo)]
    lib.dt_destroy_plan.argtypes = [vp]
    lib.dt_distance.argtypes = [vp, vp, i64, vp, vp]
    lib.dt_gradient.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.dt_hessian.argtypes = [vp, vp, i64, vp, vp]
    lib.dt_sign.argtypes = [vp, ctypes.POINTER(DtShape), vp, vp, vp]
    lib.dt_forward.argtypes = [vp, vp, i64, ctypes.POINTER(DtShape), ctypes.POINTER(DtOutputs), vp]
    lib.dt_backward.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    lib.dt_last_error.argtypes = [vp]
    lib.dt_last_stats.argtypes = [vp, ctypes.POINTER(DtCallStats)]
    lib.dt_plan_set_timing.argtypes = [vp, ctypes.c_int]
    lib.dt_plan_timings.argtypes = [vp, ctypes.POINTER(DtPassTiming), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.dt_plan_reset_timings.argtypes = [vp]
    lib.dt_create_batch_plan.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(DtInstanceDesc),
                                         ctypes.c_int, ctypes.c_uint, dbl]
    lib.dt_batch_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.dt_batch_set_workspace.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.dt_batch_instance_info.argtypes = [vp, ctypes.c_int, ctypes.POINTER(DtBatchInstanceInfo)]
    lib.dt_batch_set_tiles.argtypes = [vp, ctypes.POINTER(DtBatchTiles)]
    lib.dt_batch_get_tiles.argtypes = [vp, ctypes.POINTER(DtBatchTiles)]
    lib.dt_batch_set_schedule.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.dt_batch_get_schedule.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.dt_batch_set_graph.argtypes = [vp, ctypes.c_int]
    lib.dt_forward_batched.argtypes = [vp, vp, ctypes.POINTER(i64), vp, vp, vp]
    lib.dt_batch_autotune.argtypes = [vp, vp, ctypes.POINTER(i64), vp, vp, ctypes.c_int, vp,
                                      ctypes.POINTER(DtBatchTiles)]
    lib.dt_batch_last_error.argtypes = [vp]
    lib.dt_batch_stats.argtypes = [vp, ctypes.c_int, ctypes.POINTER(DtCallStats)]
    lib.dt_destroy_batch_plan.argtypes = [vp]
    lib.dt_status_str.argtypes = [st]
    lib.dt_status_str.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name != "dt_status_str":
            getattr(lib, name).restype = st
    _lib = lib
    return lib


def status_str(status):
    try:
        return load().dt_status_str(int(status)).decode()
    except ImportError:
        return f"status {status}"


def check(status, where):
    if status != DT_OK:
        raise DtError(status, where)
