"""Pins of the model's components against a brute-force splat renderer.

The renderer (oracle/splat_render.py) alpha-blends exact per-ray Gaussian
peaks (Eq. 11) without the EWA approximation.  Finite differences of its
image pin, component by component, what the scoring assumes:
visibility V = alpha * T with T = 1 as the unoccluded upper bound (Eq. 12),
the 1/z^2 depth law of the projection term (Eq. 14-17), the projected
covariance Sigma' and Jacobian J (Eq. 14), and the visibility gate.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import splat_render as sr
from tests.helpers import CLAMP_K, E_COL, E_LNGEM, E_OPA, ETA, Z_NEAR, camera, raw_prim


def P(**kw):
    import oracle
    base = dict(eta=ETA, z_near=Z_NEAR, clamp_k=CLAMP_K, e_col=E_COL, e_opa=E_OPA, e_lngem=E_LNGEM)
    base.update(kw)
    return oracle.Params(**base)


def _pair(mu, rot, scale, opacity):
    """The same primitive for the oracle (raw float32 values) and the renderer
    (physical values recomputed from those float32 values)."""
    x, y, z, w = rot.as_quat()
    ls = np.log(np.asarray(scale, dtype=np.float64)).astype(np.float32)
    logit = np.float32(math.log(opacity / (1.0 - opacity)))
    raw = raw_prim(mu=mu, log_scale=ls, quat=(w, x, y, z), logit=logit)
    qf = raw[6:10].astype(np.float64)
    g = sr.Gaussian(mu=raw[0:3].astype(np.float64),
                    rot=Rotation.from_quat([qf[1], qf[2], qf[3], qf[0]]).as_matrix(),
                    scale=np.exp(ls.astype(np.float64)),
                    opacity=1.0 / (1.0 + math.exp(-float(logit))),
                    color=np.array([0.6, 0.3, 0.2]))
    return raw, g


def _cam(cam18):
    c = cam18.astype(np.float64)
    return sr.Camera(R=c[:9].reshape(3, 3), t=c[9:12], fx=c[12], fy=c[13], cx=c[14], cy=c[15],
                     W=int(c[16]), H=int(c[17]))


def test_visibility_is_alpha_without_occlusion(oracle_lib):
    cam18 = camera(W=96, H=72, cx=48.0, cy=36.0, fx=200.0, fy=200.0)
    for op in (0.2, 0.5, 0.9):
        _, g = _pair((0.05, -0.03, 2.0), Rotation.from_euler("z", 30, degrees=True),
                     (0.08, 0.05, 0.06), op)
        fd = sr.fd_color_grad([g], _cam(cam18), 0)
        _, dens = sr.render([g], _cam(cam18))
        m = dens[0] > 1e-3
        np.testing.assert_allclose(fd[m] / dens[0][m], g.opacity, rtol=1e-7)


def test_occlusion_only_lowers_visibility(oracle_lib):
    """With an occluder in front, dC/dc = alpha G T <= alpha G: the zero-
    occlusion value V = alpha is an upper bound (Eq. 12, T = 1)."""
    cam18 = camera(W=96, H=72, cx=48.0, cy=36.0, fx=200.0, fy=200.0)
    _, back = _pair((0.0, 0.0, 3.0), Rotation.identity(), (0.1, 0.1, 0.1), 0.7)
    _, front = _pair((0.02, 0.0, 1.5), Rotation.identity(), (0.05, 0.05, 0.05), 0.8)
    cam = _cam(cam18)
    fd = sr.fd_color_grad([back, front], cam, 0)
    _, dens = sr.render([back, front], cam)
    bound = back.opacity * dens[0]
    assert np.all(fd <= bound + 1e-9)
    assert fd.sum() < 0.9 * bound.sum()          # the occluder removes a visible share
    fd_alone = sr.fd_color_grad([back], cam, 0)
    np.testing.assert_allclose(fd_alone, bound, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("mode", [0, 1])
def test_depth_law_of_projection_term(oracle_lib, mode):
    """Colour-gradient energy of a fixed 3D Gaussian falls as 1/z^2 (its
    footprint area); the oracle's projection term follows (Eq. 17)."""
    cam18 = camera(W=200, H=160, cx=100.0, cy=80.0, fx=400.0, fy=400.0)
    cam = _cam(cam18)
    rot = Rotation.from_euler("xyz", [20, 40, 10], degrees=True)
    energies, Ps = [], []
    for z in (2.0, 4.0):
        raw, g = _pair((0.0, 0.0, z), rot, (0.06, 0.03, 0.04), 0.6)
        fd = sr.fd_color_grad([g], cam, 0)
        energies.append(float((fd ** 2).sum()))
        Ps.append(oracle_lib.pair(raw, cam18, P(proj_mode=mode))[2]["P"])
    ratio_render = energies[0] / energies[1]
    ratio_oracle = Ps[0] / Ps[1]
    assert abs(ratio_render / 4.0 - 1.0) < 0.05
    assert abs(ratio_oracle / ratio_render - 1.0) < 0.05


@pytest.mark.parametrize("seed", range(4))
def test_projected_covariance_matches_rendered_footprint(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    rot = Rotation.random(random_state=seed)
    scale = rng.uniform(0.02, 0.06, size=3)
    cam18 = camera(W=160, H=120, cx=80.0, cy=60.0, fx=300.0, fy=280.0)
    raw, g = _pair((rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), 2.0), rot, scale, 0.5)
    _, dens = sr.render([g], _cam(cam18))
    _, cen, mom = sr.footprint_moments(dens[0])
    _, _, d = oracle_lib.pair(raw, cam18, P())
    S = np.array([[d["a"], d["b"]], [d["b"], d["c"]]])
    np.testing.assert_allclose(mom, S, rtol=2e-2, atol=2e-2 * np.abs(S).max())
    # perspective shifts the footprint's centroid off Pi(mu) at second order,
    # by about (sigma / z) times the footprint's pixel std
    shift = (scale.max() / 2.0) * math.sqrt(max(d["a"], d["c"]))
    np.testing.assert_allclose(cen, [d["u"], d["v"]], atol=1.5 * shift)
    np.testing.assert_allclose(np.unravel_index(dens[0].argmax(), dens[0].shape)[::-1],
                               [d["u"] - 0.5, d["v"] - 0.5], atol=0.75)


def test_centre_jacobian_matches_rendered_footprint(oracle_lib):
    """d(projected centre)/d(mu) = J W (Eq. 13-14), from the renderer."""
    Rv = Rotation.from_euler("xyz", [5, -10, 15], degrees=True).as_matrix()
    t = np.array([0.1, -0.05, 2.5])
    cam18 = camera(R=Rv, t=t, W=160, H=120, cx=80.0, cy=60.0, fx=300.0, fy=260.0)
    raw, g = _pair((0.1, 0.05, -0.1), Rotation.from_euler("y", 25, degrees=True), (0.03, 0.02, 0.025), 0.5)
    Jfd = sr.fd_centroid_jacobian(g, _cam(cam18), h=1e-4)
    _, _, d = oracle_lib.pair(raw, cam18, P())
    JW = d["J"] @ cam18[:9].astype(np.float64).reshape(3, 3)
    np.testing.assert_allclose(Jfd, JW, rtol=1e-2, atol=1e-2 * np.abs(JW).max())


def test_gate_matches_renderer_for_invisible_primitives(oracle_lib):
    cam18 = camera(W=96, H=72, cx=48.0, cy=36.0, fx=200.0, fy=200.0)
    cam = _cam(cam18)
    # far to the side of the image, and behind the camera
    for mu in ((6.0, 0.0, 2.0), (0.0, 0.0, -2.0)):
        raw, g = _pair(mu, Rotation.identity(), (0.05, 0.05, 0.05), 0.9)
        fd = sr.fd_color_grad([g], cam, 0)
        assert np.abs(fd).max() < 1e-30
        assert oracle_lib.pair(raw, cam18, P())[0] == 0
    # in view: both see it
    raw, g = _pair((0.0, 0.0, 2.0), Rotation.identity(), (0.05, 0.05, 0.05), 0.9)
    assert np.abs(sr.fd_color_grad([g], cam, 0)).max() > 0.1
    assert oracle_lib.pair(raw, cam18, P())[0] == 1
