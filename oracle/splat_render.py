"""Brute-force FP64 Gaussian splat renderer -- TEST INFRASTRUCTURE ONLY.

Renders a handful of 3D Gaussians into a tiny image by front-to-back alpha
blending (Eq. 11 of the paper): C(p) = sum_i c_i * alpha_i * G_i(p) * T_i(p)
with T_i(p) = prod_{j<i} (1 - alpha_j G_j(p)).

It deliberately avoids the EWA local-affine projection that the scoring
approximates: G_i(p) is the exact peak of the 3D Gaussian along the pixel's
viewing ray, exp(-q*/2) with q* = min_t (o + t d - mu)^T Sigma^-1 (o + t d - mu),
so comparing the two tests the approximation rather than restating it.
Primitives are given directly by centre, 3x3 rotation matrix, scales,
opacity in [0, 1] and an RGB colour; no quaternion or activation code.

The finite-difference helpers differentiate the rendered image with respect
to one primitive's colour or centre, the quantities the Hessian-field model
(Eq. 8, 9) is built from.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Gaussian:
    mu: np.ndarray           # (3,) world centre
    rot: np.ndarray          # (3, 3) rotation; columns are the principal axes
    scale: np.ndarray        # (3,) standard deviations along the axes
    opacity: float           # in [0, 1]
    color: np.ndarray        # (3,)


@dataclasses.dataclass
class Camera:
    R: np.ndarray            # (3, 3) world-to-camera rotation
    t: np.ndarray            # (3,)
    fx: float
    fy: float
    cx: float
    cy: float
    W: int
    H: int


def pixel_rays(cam: Camera):
    """World-space origin and (unnormalised, camera-z = 1) ray directions of
    every pixel centre, shape (H, W, 3)."""
    jj, ii = np.meshgrid(np.arange(cam.W) + 0.5, np.arange(cam.H) + 0.5)
    dc = np.stack([(jj - cam.cx) / cam.fx, (ii - cam.cy) / cam.fy, np.ones_like(jj)], axis=-1)
    dw = dc @ cam.R            # R^T d for each pixel (row-vector form)
    origin = -cam.R.T @ cam.t
    return origin, dw


def peak_density(g: Gaussian, origin, dirs):
    """exp(-q*/2) along each ray, 0 where the peak lies behind the camera."""
    inv = g.rot @ np.diag(1.0 / g.scale ** 2) @ g.rot.T
    m = g.mu - origin
    Ad = dirs @ inv                               # (H, W, 3)
    dAd = np.einsum("hwk,hwk->hw", Ad, dirs)
    dAm = Ad @ m
    mAm = m @ inv @ m
    q = mAm - dAm ** 2 / dAd
    tstar = dAm / dAd
    return np.where(tstar > 0.0, np.exp(-0.5 * np.maximum(q, 0.0)), 0.0)


def render(gaussians, cam: Camera):
    """RGB image (H, W, 3) and per-primitive peak density maps (n, H, W)."""
    origin, dirs = pixel_rays(cam)
    depth = [float(cam.R[2] @ g.mu + cam.t[2]) for g in gaussians]
    order = np.argsort(depth, kind="stable")
    img = np.zeros((cam.H, cam.W, 3))
    T = np.ones((cam.H, cam.W))
    dens = np.zeros((len(gaussians), cam.H, cam.W))
    for i in order:
        g = gaussians[i]
        if depth[i] <= 0.0:
            continue
        G = peak_density(g, origin, dirs)
        dens[i] = G
        a = g.opacity * G
        img += (a * T)[..., None] * np.asarray(g.color)[None, None, :]
        T = T * (1.0 - a)
    return img, dens


def fd_color_grad(gaussians, cam: Camera, i: int, h: float = 1e-4):
    """Central difference of the red channel w.r.t. primitive i's red colour."""
    def img_with(delta):
        gs = [dataclasses.replace(g) for g in gaussians]
        c = np.array(gs[i].color, dtype=np.float64)
        c[0] += delta
        gs[i] = dataclasses.replace(gs[i], color=c)
        return render(gs, cam)[0][..., 0]
    return (img_with(h) - img_with(-h)) / (2.0 * h)


def footprint_moments(density: np.ndarray):
    """Mass, centroid (u, v) and second central moments [[uu, uv], [uv, vv]]
    of a density map sampled at pixel centres."""
    H, W = density.shape
    jj, ii = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    m = density.sum()
    cu = (density * jj).sum() / m
    cv = (density * ii).sum() / m
    uu = (density * (jj - cu) ** 2).sum() / m
    vv = (density * (ii - cv) ** 2).sum() / m
    uv = (density * (jj - cu) * (ii - cv)).sum() / m
    return m, np.array([cu, cv]), np.array([[uu, uv], [uv, vv]])


def fd_centroid_jacobian(g: Gaussian, cam: Camera, h: float = 1e-4):
    """d(centroid)/d(mu) (2x3) of one primitive's rendered footprint."""
    J = np.zeros((2, 3))
    origin, dirs = pixel_rays(cam)
    for k in range(3):
        cs = []
        for sgn in (1.0, -1.0):
            mu = np.array(g.mu, dtype=np.float64)
            mu[k] += sgn * h
            d = peak_density(dataclasses.replace(g, mu=mu), origin, dirs)
            cs.append(footprint_moments(d)[1])
        J[:, k] = (cs[0] - cs[1]) / (2.0 * h)
    return J
