"""ctypes front end of ``refine_oracle.c`` -- TEST INFRASTRUCTURE ONLY.

Thin argument marshalling: every number is computed by the C oracle in
double precision.  ``build()`` compiles the shared library with gcc (no
fast-math, no FMA contraction, IEEE double throughout).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "refine_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so``."""
    global _lib
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    _lib = None
    return _LIB


class _CParams(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("z_near", ctypes.c_double), ("clamp_k", ctypes.c_double),
                ("e_col", ctypes.c_double), ("e_opa", ctypes.c_double), ("e_lngem", ctypes.c_double),
                ("proj_mode", ctypes.c_int32), ("vis_mode", ctypes.c_int32),
                ("equal_lambda", ctypes.c_int32), ("n_sub_views", ctypes.c_int32),
                ("amb_k", ctypes.c_double), ("score_kind", ctypes.c_int32)]


@dataclasses.dataclass
class Params:
    """Method constants and switches.

    eta: stability constant of Eq. (17) (0.05 in the paper), reused in
    Eq. (features) and Eq. (18).  z_near, clamp_k: visibility gate and EWA
    Jacobian clamp (readings).  e_col, e_opa, e_lngem: the calibration
    expectations of Eq. (18), here the expectations of the features under
    the synthetic scene distribution (reading).  proj_mode 0/1/2: projected-
    covariance energy / Eq. (17) depth term / no projection term.
    vis_mode 0/1: V = alpha / V = 1.  equal_lambda: lambda^k = 1/3.
    n_sub_views: 0 = every view, m = views floor(j V / m).
    amb_k: width of the FP32-reach bands of the gate decisions, in units of
    the FP32 roundoff 2^-24 times each decision's error magnitude (the
    bounds are derived in refine_oracle.c, above pair_eval).
    score_kind: 0 = importance score (Eq. 7 with Eq. 20), 1 = the opacity-only
    ranking of the introduction's parameter-space baseline (D = alpha).
    """

    eta: float = 0.05
    z_near: float = 0.2
    clamp_k: float = 1.3
    e_col: float = 8.892106e-3
    e_opa: float = 0.1767277
    e_lngem: float = -0.4890595
    proj_mode: int = 0
    vis_mode: int = 0
    equal_lambda: int = 0
    n_sub_views: int = 0
    amb_k: float = 16.0
    score_kind: int = 0

    def c(self) -> _CParams:
        return _CParams(self.eta, self.z_near, self.clamp_k, self.e_col, self.e_opa, self.e_lngem,
                        self.proj_mode, self.vis_mode, self.equal_lambda, self.n_sub_views,
                        self.amb_k, self.score_kind)


def load():
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.oracle_nonfinite.argtypes = [P, i64, i64]
    lib.oracle_nonfinite.restype = i64
    lib.oracle_stats.argtypes = [P, i64, i64, ctypes.c_double, P]
    lib.oracle_stats.restype = None
    lib.oracle_lambda.argtypes = [P, ctypes.POINTER(_CParams), P]
    lib.oracle_lambda.restype = None
    lib.oracle_pair.argtypes = [P, P, ctypes.POINTER(_CParams), P, P]
    lib.oracle_pair.restype = ctypes.c_int
    lib.oracle_activate.argtypes = [P, P]
    lib.oracle_activate.restype = None
    lib.oracle_score.argtypes = [P, i64, i64, P, ctypes.c_int32, ctypes.POINTER(_CParams), P, P, i64,
                                 P, P, P, P]
    lib.oracle_score.restype = None
    lib.oracle_n_prune.argtypes = [i64, ctypes.c_double]
    lib.oracle_n_prune.restype = i64
    lib.oracle_select.argtypes = [P, i64, i64, P, P]
    lib.oracle_select.restype = None
    lib.oracle_compact.argtypes = [P, i64, i64, P, P, i64, P]
    lib.oracle_compact.restype = i64
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _planes(planes: np.ndarray, n: int | None):
    planes = np.ascontiguousarray(planes, dtype=np.float32)
    if planes.ndim != 2 or planes.shape[0] != 59:
        raise ValueError("planes must be [59][stride]")
    stride = planes.shape[1]
    n = stride if n is None else int(n)
    if n > stride:
        raise ValueError("n > stride")
    return planes, n, stride


def nonfinite(planes, n=None) -> int:
    planes, n, stride = _planes(planes, n)
    return int(load().oracle_nonfinite(_ptr(planes), n, stride))


def stats(planes, n=None, eta: float = 0.05) -> dict:
    """Scene features of Eq. (features)."""
    planes, n, stride = _planes(planes, n)
    out = np.zeros(4, dtype=np.float64)
    load().oracle_stats(_ptr(planes), n, stride, float(eta), _ptr(out))
    return {"ybar": out[0], "f_col": out[1], "f_opa": out[2], "f_gem": out[3]}


def lam(F: dict, prm: Params | None = None) -> np.ndarray:
    """Content-adaptive weights {gem, col, opa} (Eq. 18, 19)."""
    prm = prm or Params()
    f = np.array([F["ybar"], F["f_col"], F["f_opa"], F["f_gem"]], dtype=np.float64)
    out = np.zeros(3, dtype=np.float64)
    cp = prm.c()
    load().oracle_lambda(_ptr(f), ctypes.byref(cp), _ptr(out))
    return out


def _cams(cams):
    cams = np.ascontiguousarray(cams, dtype=np.float32)
    if cams.ndim != 2 or cams.shape[1] != 18:
        raise ValueError("cams must be [V][18]")
    return cams


def pair(prim14, cam18, prm: Params | None = None):
    """One (primitive, view) evaluation: returns (g, amb_bits, dict)."""
    prm = prm or Params()
    p = np.ascontiguousarray(prim14, dtype=np.float32).reshape(14)
    c = np.ascontiguousarray(cam18, dtype=np.float32).reshape(18)
    out = np.zeros(20, dtype=np.float64)
    amb = np.zeros(1, dtype=np.int32)
    cp = prm.c()
    g = load().oracle_pair(_ptr(p), _ptr(c), ctypes.byref(cp), _ptr(out), _ptr(amb))
    d = {"x": out[0], "y": out[1], "z": out[2], "u": out[3], "v": out[4],
         "J": out[5:11].reshape(2, 3).copy(), "a": out[11], "b": out[12], "c": out[13],
         "r": out[14], "P": out[15], "m": out[16], "band_x": out[17], "band_y": out[18],
         "band_z": out[19]}
    return int(g), int(amb[0]), d


def activate_one(prim14) -> dict:
    p = np.ascontiguousarray(prim14, dtype=np.float32).reshape(14)
    out = np.zeros(18, dtype=np.float64)
    load().oracle_activate(_ptr(p), _ptr(out))
    return {"s": out[0:3].copy(), "sbar2": out[3], "alpha": out[4], "Y": out[5],
            "gt_gem": out[6], "gt_col": out[7], "gt_opa": out[8], "R": out[9:18].reshape(3, 3).copy()}


def score(planes, cams, lam_, prm: Params | None = None, n=None, idx=None):
    """Scores of all primitives (or of ``idx``): returns (D, D_lo, D_hi, n_amb)."""
    prm = prm or Params()
    planes, n, stride = _planes(planes, n)
    cams = _cams(cams)
    lam_ = np.ascontiguousarray(lam_, dtype=np.float64).reshape(3)
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        if idx.size and (idx.min() < 0 or idx.max() >= n):
            raise IndexError("idx out of range")
        m = idx.size
    else:
        m = n
    D = np.zeros(m, dtype=np.float64)
    lo = np.zeros(m, dtype=np.float64)
    hi = np.zeros(m, dtype=np.float64)
    na = np.zeros(m, dtype=np.int32)
    cp = prm.c()
    load().oracle_score(_ptr(planes), n, stride, _ptr(cams), cams.shape[0], ctypes.byref(cp),
                        _ptr(lam_), _ptr(idx) if idx is not None else None, m,
                        _ptr(D), _ptr(lo), _ptr(hi), _ptr(na))
    return D, lo, hi, na


def num_threads() -> int:
    return int(load().oracle_num_threads())


def n_prune(n: int, ratio: float) -> int:
    return int(load().oracle_n_prune(int(n), float(ratio)))


def select(D, n_prune_: int):
    """Keep mask (uint8) and ranking of the global sort of Sec. 3.3."""
    D = np.ascontiguousarray(D, dtype=np.float64)
    n = D.size
    keep = np.zeros(n, dtype=np.uint8)
    order = np.zeros(n, dtype=np.int64)
    load().oracle_select(_ptr(D), n, int(n_prune_), _ptr(keep), _ptr(order))
    return keep, order


def compact(planes, keep, n=None):
    """Survivor planes [59][n_keep] and index map."""
    planes, n, stride = _planes(planes, n)
    keep = np.ascontiguousarray(keep, dtype=np.uint8)
    if keep.size < n:
        raise ValueError("keep shorter than n")
    k = int(keep[:n].astype(bool).sum())
    out = np.zeros((59, max(k, 1)), dtype=np.float32)
    idx = np.zeros(max(k, 1), dtype=np.int32)
    got = load().oracle_compact(_ptr(planes), n, stride, _ptr(keep), _ptr(out), out.shape[1], _ptr(idx))
    assert got == k
    return out[:, :k], idx[:k]
