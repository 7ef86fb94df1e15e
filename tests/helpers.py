"""Shared test helpers: parameter values both sides receive, scene builders
for hand-made primitives, and the parity comparison rules.

The method constants are spelled out here once and handed to the oracle and
to the GPU library separately, so neither side's defaults feed the other.
"""
from __future__ import annotations

import math

import numpy as np

# Constants of the method as read from the paper (eta of Eq. 17) and the
# readings of its unstated parts (gate, clamp, calibration expectations).
ETA = 0.05
Z_NEAR = 0.2
CLAMP_K = 1.3
E_COL = 8.892106e-3
E_OPA = 0.1767277
E_LNGEM = -0.4890595

# Parity tolerance on scores: |D_gpu - D_ref| <= max(REL * |D_ref|, ABS).
REL_TOL = 1e-4
ABS_TOL = 1e-7

SH_C0 = 1.0 / (2.0 * math.sqrt(math.pi))   # band-0 real SH basis value


def raw_prim(mu=(0.0, 0.0, 5.0), log_scale=(-3.0, -3.0, -3.0), quat=(1.0, 0.0, 0.0, 0.0),
             logit=0.0, dc=(0.0, 0.0, 0.0)):
    """14 raw values of one primitive in plane order."""
    return np.array(list(mu) + list(log_scale) + list(quat) + [logit] + list(dc), dtype=np.float32)


def planes_from_prims(prims, stride=None):
    """[59][stride] planes from a list of 14-value primitives (SH rest = 0)."""
    n = len(prims)
    stride = n if stride is None else stride
    out = np.zeros((59, max(stride, 1)), dtype=np.float32)[:, :stride]
    for i, p in enumerate(prims):
        out[:14, i] = p
    return np.ascontiguousarray(out)


def camera(R=np.eye(3), t=(0.0, 0.0, 0.0), fx=300.0, fy=300.0, cx=160.0, cy=120.0, W=320, H=240):
    row = np.zeros(18, dtype=np.float64)
    row[0:9] = np.asarray(R, dtype=np.float64).reshape(9)
    row[9:12] = t
    row[12:18] = (fx, fy, cx, cy, W, H)
    return row.astype(np.float32)


def within_interval(d_gpu, lo, hi, rel=REL_TOL, abs_=ABS_TOL):
    """True where d_gpu lies in [lo - tol, hi + tol], tol from the bound."""
    d_gpu = np.asarray(d_gpu, dtype=np.float64)
    tol_lo = np.maximum(rel * np.abs(lo), abs_)
    tol_hi = np.maximum(rel * np.abs(hi), abs_)
    return (d_gpu >= lo - tol_lo) & (d_gpu <= hi + tol_hi)
