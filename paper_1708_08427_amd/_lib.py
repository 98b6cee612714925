"""ctypes declarations of the C ABI in include/hq.h (libhq.so)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhq.so")

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_vp = ctypes.c_void_p
P_i32 = ctypes.POINTER(ctypes.c_int32)
P_i64 = ctypes.POINTER(ctypes.c_int64)
P_f64 = ctypes.POINTER(ctypes.c_double)

HQ_OK, HQ_E_INVALID, HQ_E_DEGENERATE, HQ_E_NOMEM, HQ_E_DEVICE, HQ_E_UNSUPPORTED = range(6)
HQ_FP64, HQ_FP32 = 0, 1
HQ_ROWS, HQ_TRIPLES = 0, 1
HQ_FLAG_NONFINITE, HQ_FLAG_STACK, HQ_FLAG_BOUNDS, HQ_FLAG_PHASES = 1, 2, 4, 8
HQ_BODY_ILLCOND, HQ_BODY_DEGENERATE = 1, 2


class Options(ctypes.Structure):
    _fields_ = [("tile_units", c_i32), ("store", c_i32), ("explicit_dense_max_n", c_i32), ("max_phases", c_i32),
                ("run_nodes", c_i32), ("waves_per_cu", c_i32), ("keep_node_data", c_i32),
                ("later_tile_units", c_i32), ("first_waves_per_cu", c_i32), ("max_nrhs", c_i32),
                ("max_tiles", c_i32), ("krylov_nrhs", c_i32),
                ("sweep_kernel", c_i32), ("fused_upward", c_i32), ("leaf_size", c_i32)]


class KrylovInfo(ctypes.Structure):
    _fields_ = [("max_iter", c_i32), ("rtol", ctypes.c_double), ("iters", c_i32),
                ("max_rel_residual", ctypes.c_double), ("check_every", c_i32)]


# int (*)(const void *x, void *y, int64_t nrhs, void *user, hq_stream stream)
DAPPLY_FN = ctypes.CFUNCTYPE(ctypes.c_int, c_vp, c_vp, c_i64, c_vp, c_vp)


class Info(ctypes.Structure):
    _fields_ = [("N", c_i64), ("m", c_i64), ("rows", c_i64), ("internal_nodes", c_i64), ("tiles", c_i64),
                ("phases", c_i32), ("device_flags", c_i32), ("tile_units", c_i32), ("store", c_i32),
                ("max_kappa", ctypes.c_double), ("ill_conditioned_bodies", c_i64), ("degenerate_bodies", c_i64)]


# (name, restype, argtypes) of every exported function
SIGNATURES = [
    ("hq_build", c_i32, [c_vp, P_i64, c_i64, ctypes.POINTER(Options), c_vp, ctypes.POINTER(c_vp)]),
    ("hq_workspace_bytes", c_i32, [P_i64, c_i64, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)]),
    ("hq_build_into", c_i32, [c_vp, P_i64, c_i64, ctypes.POINTER(Options), c_vp, ctypes.c_size_t, c_vp,
                              ctypes.POINTER(c_vp)]),
    ("hq_autotune", c_i32, [c_vp, P_i64, c_i64, c_i64, c_i32, c_i32, ctypes.c_int, ctypes.POINTER(Options), c_vp,
                            ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_double)]),
    ("hq_rebuild", c_i32, [c_vp, c_vp, c_vp]),
    ("hq_reserve", c_i32, [c_vp, c_i64, c_i32]),
    ("hq_apply", c_i32, [c_vp, c_vp, c_vp, ctypes.c_int, c_i64, c_i32, c_vp]),
    ("hq_apply_layout", c_i32, [c_vp, c_vp, c_vp, ctypes.c_int, c_i64, c_i32, c_i32, c_vp]),
    ("hq_apply_noalloc", c_i32, [c_vp, c_vp, c_vp, ctypes.c_int, c_i64, c_i32, c_i32, c_vp]),
    ("hq_apply_full", c_i32, [c_vp, c_vp, c_vp, c_vp, ctypes.c_int, c_i64, c_i32, c_i32, c_vp]),
    ("hq_apply_rotated", c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.c_int, c_i64, c_i32, c_i32, c_vp]),
    ("hq_constrained_solve", c_i32, [c_vp, DAPPLY_FN, c_vp, c_vp, c_vp, c_vp, c_i64, c_i32, c_i32, c_vp, c_vp,
                                     ctypes.POINTER(KrylovInfo), c_vp]),
    ("hq_apply_timed", c_i32, [c_vp, c_vp, c_vp, ctypes.c_int, c_i64, c_i32, c_i32, c_vp,
                               ctypes.POINTER(ctypes.c_float), c_i32, P_i32]),
    ("hq_stream_ceiling", c_i32, [c_vp, ctypes.c_size_t, c_vp, ctypes.c_size_t, c_i32, c_vp, c_vp]),
    ("hq_node_phase", c_i32, [c_vp, P_i32]),
    ("hq_explicit", c_i32, [c_vp, c_i64, c_vp, c_i64, c_vp]),
    ("hq_explicit_blocks_size", c_i32, [c_vp, c_i64, P_i64, P_i64]),
    ("hq_explicit_blocks", c_i32, [c_vp, c_i64, c_i32, c_vp, P_i64, P_i64, P_i64, P_i32, P_i32, c_vp]),
    ("hq_sorted_beads", c_i32, [c_vp, c_i64, P_i64]),
    ("hq_rigid_update", c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    ("hq_rigid_motion", c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    ("hq_query", c_i32, [c_vp, ctypes.POINTER(Info)]),
    ("hq_body_info", c_i32, [c_vp, P_i32, P_f64]),
    ("hq_node_data", c_i32, [c_vp, P_i32, P_i32, P_i32, P_i32, P_i32, P_i32, P_f64, P_f64, P_f64, P_i32, P_i32]),
    ("hq_capture_begin", c_i32, [c_vp]),
    ("hq_capture_end", c_i32, [c_vp, ctypes.POINTER(c_vp)]),
    ("hq_graph_launch", c_i32, [c_vp, c_vp]),
    ("hq_graph_destroy", None, [c_vp]),
    ("hq_destroy", None, [c_vp]),
    ("hq_status_string", ctypes.c_char_p, [c_i32]),
    ("hq_last_error", ctypes.c_char_p, []),
]

_lib = None


def load(path: str | None = None):
    """Load libhq.so.  There is no fallback: a missing library is an error."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(p)
    for name, res, args in SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib
