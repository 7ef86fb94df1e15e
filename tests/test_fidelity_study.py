"""The approximation-fidelity study (research context, not parity) on a
tiny scene: its finite differences reproduce the exact removal identity,
its DER is 1 where primitives cannot interact, and the REFINE ranking is
positively associated with the true removal error."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from tests import fidelity as fd


def test_study_small_scene():
    r = fd.study(n=16, V=4, seed=0, neighbourhoods=1, k_nn=6)
    # removing i changes the image by exactly -alpha_i dR/dalpha_i (multilinear blending)
    assert r["removal_identity_max_rel_err"] < 1e-5
    assert 0.0 < r["der_primitives"] <= 1.0 and 0.0 < r["der_attributes"] <= 1.0
    assert r["spearman_D_cov_vs_removal"] > 0.3
    # REFINE's weight (alpha S / |V|) ranks like the exact diagonal weights of
    # the scale and colour groups, which scale with alpha as it does
    assert r["spearman_w_vs_exact_diag_gem"] > 0.3 and r["spearman_w_vs_exact_diag_col"] > 0.3
    assert -1.0 <= r["spearman_w_vs_exact_diag_opa"] <= 1.0


def test_exact_opacity_weight_is_the_removal_error_over_alpha_squared():
    """Blending is multilinear in the opacities, so removing i changes the
    image by exactly -alpha_i dR/dalpha_i: the exact opacity weight (from the
    finite differences in the logit and the chain rule) is Q_i / alpha_i^2."""
    prims = fd.make_scene(10, seed=4)
    rows, cams = fd.make_cameras(3)
    caches = [fd.ViewCache(prims, c) for c in cams]
    W = fd.exact_group_weights(prims, caches)
    Q = fd.removal_errors(prims, caches)
    alpha = np.array([1.0 / (1.0 + math.exp(-p.logit)) for p in prims])
    seen = Q > 1e-12
    assert seen.sum() >= 5
    np.testing.assert_allclose(W["opa"][seen], Q[seen] / alpha[seen] ** 2, rtol=1e-5)


def test_der_is_one_for_separated_primitives():
    prims = [fd.Prim(mu=np.array([0.0, y, z]), log_scale=np.full(3, math.log(0.05)), rot=np.eye(3), logit=0.5,
                     dc=np.array([0.2, -0.1, 0.3])) for y in (-0.8, 0.8) for z in (-0.4, 0.4)]
    rows, cams = fd.make_cameras(1)
    caches = [fd.ViewCache(prims, c) for c in cams]
    H = fd.gauss_newton(fd.jacobian(prims, caches, list(range(4))))
    assert fd.der_primitives(H, 4) > 1.0 - 1e-9
    # the cached compositing equals the renderer's own image
    img, _ = fd.sr.render([p.gaussian() for p in prims], cams[0])
    np.testing.assert_allclose(caches[0].image(), img, rtol=0, atol=1e-12)


def test_rotation_perturbation_is_a_rotation():
    p = fd.make_scene(1, seed=3)[0]
    q = p.perturbed(7, 0.3)
    np.testing.assert_allclose(q.rot @ q.rot.T, np.eye(3), atol=1e-12)
    np.testing.assert_allclose(Rotation.from_matrix(q.rot @ p.rot.T).as_rotvec(), [0.0, 0.3, 0.0], atol=1e-12)
