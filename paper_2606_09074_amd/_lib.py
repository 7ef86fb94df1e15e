"""ctypes loader of ``librefine.so`` and mirrors of the C-ABI structures.

Argument marshalling only.  Importing this module does not touch the GPU;
loading the library fails loudly (``RuntimeError``) when it has not been
built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librefine.so")

REFINE_OK = 0
REFINE_E_INVALID = -1
REFINE_E_UNSUPPORTED = -2
REFINE_E_WORKSPACE = -3
REFINE_E_HIP = -4

REFINE_F32, REFINE_BF16, REFINE_F16 = 0, 1, 2
PROJ_COV, PROJ_DEPTH, PROJ_NONE = 0, 1, 2
VIS_ALPHA, VIS_NONE = 0, 1
PATH_AUTO, PATH_DIRECT, PATH_BINNED = 0, 1, 2
SCORE_IMPORTANCE, SCORE_OPACITY = 0, 1

EXPORTED = ("refine_version", "refine_status_string", "refine_params_default", "refine_prune_count",
            "refine_workspace_size", "refine_stats", "refine_score", "refine_score_prepare", "refine_score_cameras",
            "refine_score_views",
            "refine_select", "refine_compact", "refine_prune_batch_workspace_size", "refine_prune_batch",
            "refine_stats_noalloc")
STATS_NOALLOC_MAX_N = 67108864
BATCH_STAGING_BYTES_PER_JOB = 256


class Scene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("stride", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("sh_dtype", ctypes.c_int32), ("planes", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("z_near", ctypes.c_double), ("clamp_k", ctypes.c_double),
                ("e_col", ctypes.c_double), ("e_opa", ctypes.c_double), ("e_lngem", ctypes.c_double),
                ("proj_mode", ctypes.c_int32), ("vis_mode", ctypes.c_int32),
                ("equal_lambda", ctypes.c_int32), ("n_sub_views", ctypes.c_int32),
                ("score_path", ctypes.c_int32), ("records_per_lane", ctypes.c_int32),
                ("views_per_iteration", ctypes.c_int32), ("score_kind", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("ybar", ctypes.c_double), ("f_col", ctypes.c_double), ("f_opa", ctypes.c_double),
                ("f_gem", ctypes.c_double), ("lam", ctypes.c_double * 3), ("n", ctypes.c_int64),
                ("n_nonfinite", ctypes.c_int64), ("bbox_min", ctypes.c_float * 3),
                ("bbox_max", ctypes.c_float * 3)]


STATS_BYTES = ctypes.sizeof(Stats)


class PruneJob(ctypes.Structure):
    _fields_ = [("scene", Scene), ("cams", ctypes.c_void_p), ("n_views", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("ratio", ctypes.c_double), ("stats", ctypes.c_void_p),
                ("scores", ctypes.c_void_p), ("keep", ctypes.c_void_p), ("n_keep", ctypes.c_void_p),
                ("out", Scene), ("index_map", ctypes.c_void_p), ("n_out", ctypes.c_void_p)]

_lib = None


class RefineError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}")


def load():
    """Load the built library (no GPU access)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_09074_amd.build` "
                           "(there is no CPU fallback)")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7)
    # as the system one the library links; whichever is loaded first serves
    # the whole process, so torch is loaded first and the library's HIP calls
    # share torch's runtime, devices and streams
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    lib.refine_version.argtypes = []
    lib.refine_version.restype = ctypes.c_char_p
    lib.refine_status_string.argtypes = [i32]
    lib.refine_status_string.restype = ctypes.c_char_p
    lib.refine_params_default.argtypes = [ctypes.POINTER(Params)]
    lib.refine_params_default.restype = None
    lib.refine_prune_count.argtypes = [i64, ctypes.c_double]
    lib.refine_prune_count.restype = i64
    lib.refine_workspace_size.argtypes = [i64, i32, ctypes.POINTER(sz)]
    lib.refine_workspace_size.restype = i32
    lib.refine_stats.argtypes = [ctypes.POINTER(Scene), ctypes.POINTER(Params), P, P, sz, P]
    lib.refine_stats.restype = i32
    lib.refine_stats_noalloc.argtypes = [ctypes.POINTER(Scene), ctypes.POINTER(Params), P, P]
    lib.refine_stats_noalloc.restype = i32
    lib.refine_score.argtypes = [ctypes.POINTER(Scene), P, i32, ctypes.POINTER(Params), P, P, P, sz, P]
    lib.refine_score.restype = i32
    lib.refine_score_prepare.argtypes = [ctypes.POINTER(Scene), P, i32, ctypes.POINTER(Params), P, P, sz, P]
    lib.refine_score_prepare.restype = i32
    lib.refine_score_views.argtypes = [ctypes.POINTER(Scene), i32, ctypes.POINTER(Params), P, P, P, P, sz, P]
    lib.refine_score_views.restype = i32
    lib.refine_select.argtypes = [P, i64, ctypes.c_double, i64, P, P, P, P, sz, P]
    lib.refine_select.restype = i32
    lib.refine_compact.argtypes = [ctypes.POINTER(Scene), P, ctypes.POINTER(Scene), P, P, P, sz, P]
    lib.refine_compact.restype = i32
    lib.refine_prune_batch_workspace_size.argtypes = [P, i32, ctypes.POINTER(Params), ctypes.POINTER(sz)]
    lib.refine_prune_batch_workspace_size.restype = i32
    lib.refine_prune_batch.argtypes = [P, i32, ctypes.POINTER(Params), P, sz, P, sz, P]
    lib.refine_prune_batch.restype = i32
    _lib = lib
    return lib


def status_string(status: int) -> str:
    try:
        return load().refine_status_string(int(status)).decode()
    except RuntimeError:
        return f"status {status}"


def check(status: int, where: str) -> None:
    if status != REFINE_OK:
        raise RefineError(status, where)


def default_params() -> Params:
    p = Params()
    load().refine_params_default(ctypes.byref(p))
    return p
