"""Pins of the oracle's activation, scene features and lambda (CPU only).

Each expected value comes from a closed form, a library routine or a
brute-force sum -- not from the oracle's own formulas.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from tests.helpers import (E_COL, E_LNGEM, E_OPA, ETA, SH_C0, planes_from_prims, raw_prim)


def _params(**kw):
    import oracle
    base = dict(eta=ETA, e_col=E_COL, e_opa=E_OPA, e_lngem=E_LNGEM)
    base.update(kw)
    return oracle.Params(**base)


def _wxyz(rot: Rotation):
    x, y, z, w = rot.as_quat()          # scipy is scalar-last
    return (w, x, y, z)


def test_rotation_matches_scipy(oracle_lib):
    rng = np.random.default_rng(5)
    for rot in Rotation.random(20, random_state=11):
        q = np.array(_wxyz(rot)) * rng.uniform(0.3, 3.0)     # unnormalised on purpose
        a = oracle_lib.activate_one(raw_prim(quat=q))
        np.testing.assert_allclose(a["R"], rot.as_matrix(), atol=2e-7)
        a_neg = oracle_lib.activate_one(raw_prim(quat=-q))
        np.testing.assert_allclose(a_neg["R"], a["R"], atol=1e-12)


def test_rotation_axis_angle_example(oracle_lib):
    th = 0.7
    q = (math.cos(th / 2), 0.0, 0.0, math.sin(th / 2))       # rotation by th about +z
    R = oracle_lib.activate_one(raw_prim(quat=q))["R"]
    np.testing.assert_allclose(R @ [1.0, 0.0, 0.0], [math.cos(th), math.sin(th), 0.0], atol=1e-7)
    assert abs(np.linalg.det(R) - 1.0) < 1e-7
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-7)


def test_zero_quaternion_is_identity(oracle_lib):
    R = oracle_lib.activate_one(raw_prim(quat=(0.0, 0.0, 0.0, 0.0)))["R"]
    np.testing.assert_array_equal(R, np.eye(3))


def test_scale_opacity_activation(oracle_lib):
    a = oracle_lib.activate_one(raw_prim(log_scale=(0.0, math.log(2.0), -1.0), logit=0.0))
    np.testing.assert_allclose(a["s"], [1.0, 2.0, math.exp(-1.0)], rtol=1e-7)
    assert a["alpha"] == 0.5
    assert abs(a["sbar2"] - (1.0 + 4.0 + math.exp(-2.0)) / 3.0) < 1e-6
    # geometry area magnitude: product of the two largest scales
    assert abs(a["gt_gem"] - 2.0) < 1e-6
    logit = 1.3
    b = oracle_lib.activate_one(raw_prim(logit=logit))
    assert abs(b["alpha"] - 1.0 / (1.0 + math.exp(-np.float32(logit)))) < 1e-15
    assert b["gt_opa"] == b["alpha"]


def test_dc_colour_constant_is_sh_band0_normalisation(oracle_lib):
    # dc = 1 on every channel: rgb = 0.5 + C0, |rgb| = sqrt(3) (0.5 + C0)
    a = oracle_lib.activate_one(raw_prim(dc=(1.0, 1.0, 1.0)))
    c0 = a["gt_col"] / math.sqrt(3.0) - 0.5
    assert abs(4.0 * math.pi * c0 * c0 - 1.0) < 1e-12    # int Y00^2 dOmega = 1
    z = oracle_lib.activate_one(raw_prim(dc=(0.0, 0.0, 0.0)))
    assert abs(z["gt_col"] - 0.5 * math.sqrt(3.0)) < 1e-15
    assert abs(z["Y"] - 0.5) < 1e-15


def test_luma_weights_bt601(oracle_lib):
    # rgb = 0.5 + C0 * dc; pick dc giving pure channel offsets
    for ch, w in enumerate((0.299, 0.587, 0.114)):
        dc = [0.0, 0.0, 0.0]
        dc[ch] = 0.5 / SH_C0
        y = oracle_lib.activate_one(raw_prim(dc=dc))["Y"]
        assert abs(y - (0.5 + w * 0.5)) < 1e-7


def test_stats_constant_colour_half_opacity_isotropic(oracle_lib):
    n = 257
    prims = [raw_prim(mu=(i, 0, 0), log_scale=(-2.0, -2.0, -2.0), logit=0.0, dc=(0.3, 0.3, 0.3))
             for i in range(n)]
    F = oracle_lib.stats(planes_from_prims(prims), eta=ETA)
    s = math.exp(-2.0)
    assert F["f_col"] < 1e-25          # zero up to the rounding of the mean
    assert F["f_opa"] == 0.25
    assert abs(F["f_gem"] - s / (s + ETA)) < 1e-13


def test_stats_two_valued_scene_closed_form(oracle_lib):
    d1, d2 = -0.4, 0.9
    prims = [raw_prim(dc=(d1, d1, d1), logit=1.0, log_scale=(-4, -3, -5)) for _ in range(100)]
    prims += [raw_prim(dc=(d2, d2, d2), logit=-1.0, log_scale=(-5, -3, -4)) for _ in range(100)]
    F = oracle_lib.stats(planes_from_prims(prims), eta=ETA)
    y1, y2 = 0.5 + SH_C0 * float(np.float32(d1)), 0.5 + SH_C0 * float(np.float32(d2))
    assert abs(F["ybar"] - 0.5 * (y1 + y2)) < 1e-14
    assert abs(F["f_col"] - (0.5 * (y1 - y2)) ** 2) < 1e-14
    e = math.exp(1.0)
    assert abs(F["f_opa"] - e / (1.0 + e) ** 2) < 1e-14      # symmetric in +-logit
    gem = math.exp(-3.0) / (math.exp(-5.0) + ETA)
    assert abs(F["f_gem"] - gem) < 1e-12


def test_stats_brute_force_fsum_and_permutation(oracle_lib):
    from paper_2606_09074_amd import synth
    pl = synth.make_planes(synth.SMALL.with_n(4000))
    F = oracle_lib.stats(pl, eta=ETA)
    # brute force from the definitions with exactly rounded sums
    s = np.exp(pl[3:6].astype(np.float64))
    alpha = 1.0 / (1.0 + np.exp(-pl[10].astype(np.float64)))
    rgb = 0.5 + SH_C0 * pl[11:14].astype(np.float64)
    Y = 0.299 * rgb[0] + 0.587 * rgb[1] + 0.114 * rgb[2]
    ybar = math.fsum(Y) / Y.size
    assert abs(F["ybar"] - ybar) < 1e-13
    assert abs(F["f_col"] - math.fsum((Y - ybar) ** 2) / Y.size) < 1e-13
    assert abs(F["f_opa"] - math.fsum(alpha * (1 - alpha)) / Y.size) < 1e-13
    assert abs(F["f_gem"] - math.fsum(s.max(0) / (s.min(0) + ETA)) / Y.size) < 1e-12
    perm = np.random.default_rng(3).permutation(pl.shape[1])
    Fp = oracle_lib.stats(np.ascontiguousarray(pl[:, perm]), eta=ETA)
    for k in F:
        assert abs(F[k] - Fp[k]) <= 1e-13 * max(1.0, abs(F[k]))


def test_stats_respects_stride_and_n(oracle_lib):
    from paper_2606_09074_amd import synth
    pl = synth.make_planes(synth.SMALL.with_n(1000), stride=1037)
    pl[:, 1000:] = 99.0          # padding must be ignored
    F = oracle_lib.stats(pl, n=1000, eta=ETA)
    F2 = oracle_lib.stats(np.ascontiguousarray(pl[:, :1000]), eta=ETA)
    assert F == F2


def test_lambda_normalised_and_calibrated(oracle_lib):
    prm = _params()
    F = {"ybar": 0.5, "f_col": 0.01, "f_opa": 0.2, "f_gem": 0.7}
    lam = oracle_lib.lam(F, prm)
    assert abs(lam.sum() - 1.0) < 1e-15
    # a scene whose features equal the calibration expectations gets equal weights
    Fc = {"ybar": 0.5, "f_col": E_COL, "f_opa": E_OPA, "f_gem": math.exp(E_LNGEM) - ETA}
    np.testing.assert_allclose(oracle_lib.lam(Fc, prm), [1 / 3] * 3, atol=1e-12)
    # doubling F_col doubles lambda~col: (1, 2, 1) / 4
    Fd = dict(Fc, f_col=2 * E_COL)
    np.testing.assert_allclose(oracle_lib.lam(Fd, prm), [0.25, 0.5, 0.25], atol=1e-12)
    assert list(oracle_lib.lam(F, _params(equal_lambda=1))) == [1 / 3, 1 / 3, 1 / 3]


def test_nonfinite_count(oracle_lib):
    prims = [raw_prim() for _ in range(10)]
    pl = planes_from_prims(prims)
    assert oracle_lib.nonfinite(pl) == 0
    pl[3, 2] = np.inf
    pl[10, 7] = np.nan
    pl[20, 5] = np.nan           # higher SH is not read by the scoring
    assert oracle_lib.nonfinite(pl) == 2
