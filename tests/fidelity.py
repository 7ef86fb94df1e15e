"""Approximation-fidelity study of the REFINE score on tiny synthetic scenes.

TEST INFRASTRUCTURE / RESEARCH CONTEXT, NOT PARITY.  CPU, FP64, built on
the brute-force renderer of oracle/splat_render.py (exact per-ray peaks,
front-to-back blending of Eq. 11) and on the oracle's scores.

What it measures, per scene:

* removal error Q_i = mean over views of ||R(G) - R(G without i)||^2, the
  image change that pruning primitive i causes (the quantity Eq. 3 models);
* the Gauss-Newton matrix H = mean_v J_v^T J_v (Eq. 3, 5) of the rendered
  images with respect to every primitive's storage parameters -- centre (3),
  log-scale (3), rotation (3 small angles), opacity logit (1), SH DC (3) --
  from central finite differences of the renderer;
* the Diagonal Energy Ratio DER = sum_i ||H_ii||_F^2 / ||H||_F^2 over
  primitive blocks (assumption 1, primitive independence) and, inside the
  blocks, over the attribute groups geometry / opacity / colour
  (assumption 2, attribute orthogonality), as in the paper's Sec. 5.4;
* Spearman rank correlations of the REFINE score D (Eq. 7, 20), in both
  projection modes, and of an opacity-only ranking, with Q;
* for each attribute group (geometry scales, colour, opacity) the exact
  diagonal Gauss-Newton weight of Eq. 8 in activated units, from the
  renderer's finite differences, and its Spearman correlation with REFINE's
  weight w_i^k = lambda^k alpha_i S_i / |V| (Eq. 20).

The image is multilinear in the opacities, so removing primitive i changes
it by exactly -alpha_i dR/dalpha_i: Q_i = alpha_i^2 mean_v ||dR/dalpha_i||^2,
the diagonal Gauss-Newton weight of the activated opacity times its square.
The study checks that identity as a self-test of its finite differences.

Run ``python -m tests.fidelity`` for the larger study (printed as JSON).
"""
from __future__ import annotations

import dataclasses
import json
import math

import numpy as np
from scipy.spatial.transform import Rotation
from scipy.stats import spearmanr

from oracle import splat_render as sr
from tests.helpers import CLAMP_K, E_COL, E_LNGEM, E_OPA, ETA, SH_C0, Z_NEAR, camera, planes_from_prims, raw_prim

N_PARAMS = 13
GROUPS = {"gem": list(range(0, 9)), "opa": [9], "col": [10, 11, 12]}


@dataclasses.dataclass
class Prim:
    """Storage parameters of one primitive (what 3DGS optimises)."""
    mu: np.ndarray
    log_scale: np.ndarray
    rot: np.ndarray          # 3x3
    logit: float
    dc: np.ndarray

    def gaussian(self) -> sr.Gaussian:
        return sr.Gaussian(mu=self.mu, rot=self.rot, scale=np.exp(self.log_scale),
                           opacity=1.0 / (1.0 + math.exp(-self.logit)), color=0.5 + SH_C0 * self.dc)

    def perturbed(self, p: int, h: float) -> "Prim":
        mu, ls, rot, logit, dc = self.mu.copy(), self.log_scale.copy(), self.rot, self.logit, self.dc.copy()
        if p < 3:
            mu[p] += h
        elif p < 6:
            ls[p - 3] += h
        elif p < 9:
            w = np.zeros(3)
            w[p - 6] = h
            rot = Rotation.from_rotvec(w).as_matrix() @ rot
        elif p == 9:
            logit += h
        else:
            dc[p - 10] += h
        return Prim(mu, ls, rot, logit, dc)


def make_scene(n: int, seed: int, n_clusters: int = 3, spread: float = 0.35, log_scale_mu: float = -2.3):
    """Clustered primitives in [-1, 1]^3 (dense, overlapping footprints)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-0.6, 0.6, size=(n_clusters, 3))
    prims = []
    for i in range(n):
        mu = centres[rng.integers(n_clusters)] + rng.normal(0.0, spread, 3)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        prims.append(Prim(mu=mu.astype(np.float32).astype(np.float64),
                          log_scale=rng.normal(log_scale_mu, 0.4, 3).astype(np.float32).astype(np.float64),
                          rot=Rotation.from_quat(q).as_matrix(),
                          logit=float(np.float32(rng.normal(0.5, 1.5))),
                          dc=rng.normal(0.0, 0.5, 3).astype(np.float32).astype(np.float64)))
    return prims


def make_cameras(V: int, radius: float = 4.0, W: int = 48, H: int = 36, f: float = 40.0):
    from paper_2606_09074_amd import synth
    rows, cams = [], []
    for k in range(V):
        a = 2 * math.pi * k / V
        eye = np.array([radius * math.cos(a), radius * math.sin(a), 0.6])
        R, t = synth.look_at(eye, (0.0, 0.0, 0.0))
        row = camera(R=R, t=t, fx=f, fy=f, cx=W / 2, cy=H / 2, W=W, H=H)
        rows.append(row)
        c = row.astype(np.float64)
        cams.append(sr.Camera(R=c[:9].reshape(3, 3), t=c[9:12], fx=c[12], fy=c[13], cx=c[14], cy=c[15], W=W, H=H))
    return np.stack(rows), cams


def oracle_planes(prims):
    raws = []
    for p in prims:
        x, y, z, w = Rotation.from_matrix(p.rot).as_quat()
        raws.append(raw_prim(mu=p.mu, log_scale=p.log_scale, quat=(w, x, y, z), logit=p.logit, dc=p.dc))
    return planes_from_prims(raws)


# ----------------------------------------------------------------- renderer

class ViewCache:
    """Per-view peak densities of every primitive, so an image with one
    primitive changed re-evaluates only that primitive's density."""

    def __init__(self, prims, cam: sr.Camera):
        self.cam = cam
        self.origin, self.dirs = sr.pixel_rays(cam)
        self.gs = [p.gaussian() for p in prims]
        self.depth = np.array([float(cam.R[2] @ g.mu + cam.t[2]) for g in self.gs])
        self.dens = np.stack([self._density(g) for g in self.gs])

    def _density(self, g):
        d = float(self.cam.R[2] @ g.mu + self.cam.t[2])
        if d <= 0.0:
            return np.zeros((self.cam.H, self.cam.W))
        return sr.peak_density(g, self.origin, self.dirs)

    def image(self, i: int = -1, g_new=None, drop: bool = False):
        """Blend all primitives (Eq. 11), optionally with primitive i replaced
        by g_new or dropped."""
        gs, dens, depth = self.gs, self.dens, self.depth.copy()
        if i >= 0 and g_new is not None:
            depth[i] = float(self.cam.R[2] @ g_new.mu + self.cam.t[2])
        img = np.zeros((self.cam.H, self.cam.W, 3))
        T = np.ones((self.cam.H, self.cam.W))
        for j in np.argsort(depth, kind="stable"):
            if depth[j] <= 0.0 or (drop and j == i):
                continue
            g = g_new if (j == i and g_new is not None) else gs[j]
            G = self._density(g) if (j == i and g_new is not None) else dens[j]
            a = g.opacity * G
            img += (a * T)[..., None] * np.asarray(g.color)[None, None, :]
            T = T * (1.0 - a)
        return img


def removal_errors(prims, caches):
    base = [c.image() for c in caches]
    return np.array([np.mean([np.sum((b - c.image(i, drop=True)) ** 2) for b, c in zip(base, caches)])
                     for i in range(len(prims))])


def jacobian(prims, caches, subset, h: float = 1e-4):
    """FD Jacobian of every view's image w.r.t. the storage parameters of the
    primitives in `subset`: array [V, pixels*3, len(subset)*13]."""
    V = len(caches)
    npx = caches[0].cam.H * caches[0].cam.W * 3
    J = np.zeros((V, npx, len(subset) * N_PARAMS))
    for a, i in enumerate(subset):
        for p in range(N_PARAMS):
            gp = prims[i].perturbed(p, h).gaussian()
            gm = prims[i].perturbed(p, -h).gaussian()
            for v, c in enumerate(caches):
                J[v, :, a * N_PARAMS + p] = ((c.image(i, gp) - c.image(i, gm)) / (2 * h)).reshape(-1)
    return J


def exact_group_weights(prims, caches, h: float = 1e-4) -> dict:
    """The exact diagonal Gauss-Newton weight of each attribute group of
    every primitive (Eq. 8 with the second derivative of the image error
    replaced by J^T J): W_i^k = mean over views of the squared norm of the
    image's derivative with respect to the group's activated attributes --
    opacity alpha, DC colour c = 0.5 + C0 dc, scales s -- from central
    finite differences in the storage parameters and the chain rule
    (d/dalpha = d/dlogit / (alpha (1 - alpha)), d/dc = d/ddc / C0,
    d/ds = d/dlog s / s)."""
    n = len(prims)
    params = {"gem": [3, 4, 5], "opa": [9], "col": [10, 11, 12]}
    W = {k: np.zeros(n) for k in params}
    for i, p in enumerate(prims):
        alpha = 1.0 / (1.0 + math.exp(-p.logit))
        s = np.exp(p.log_scale)
        for k, ps in params.items():
            for q in ps:
                gp = p.perturbed(q, h).gaussian()
                gm = p.perturbed(q, -h).gaussian()
                d2 = np.mean([np.sum(((c.image(i, gp) - c.image(i, gm)) / (2 * h)) ** 2) for c in caches])
                if k == "opa":
                    d2 /= (alpha * (1.0 - alpha)) ** 2
                elif k == "col":
                    d2 /= SH_C0 ** 2
                else:
                    d2 /= s[q - 3] ** 2
                W[k][i] += d2
    return W


def refine_group_weight(prims, D, lam):
    """REFINE's weight w_i^k = lambda^k alpha_i S_i / |V| (Eq. 20) without
    its constant lambda^k: D_i / K_i with K_i = sum_k lambda^k G~_i^k
    (Eq. 7), from the oracle's scores."""
    K = []
    for p in prims:
        s = np.exp(p.log_scale)
        alpha = 1.0 / (1.0 + math.exp(-p.logit))
        g_gem = max(s[0] * s[1], s[0] * s[2], s[1] * s[2])
        g_col = float(np.linalg.norm(0.5 + SH_C0 * p.dc))
        K.append(lam[0] * g_gem + lam[1] * g_col + lam[2] * alpha)
    return np.asarray(D) / np.asarray(K)


def gauss_newton(J):
    """H = mean over views of J_v^T J_v (Eq. 3, 5 up to the noise scale)."""
    return np.einsum("vpa,vpb->ab", J, J) / J.shape[0]


def der_primitives(H, m: int) -> float:
    diag = sum(np.sum(H[a * N_PARAMS:(a + 1) * N_PARAMS, a * N_PARAMS:(a + 1) * N_PARAMS] ** 2) for a in range(m))
    return float(diag / np.sum(H ** 2))


def der_attributes(H, m: int) -> float:
    num = den = 0.0
    for a in range(m):
        B = H[a * N_PARAMS:(a + 1) * N_PARAMS, a * N_PARAMS:(a + 1) * N_PARAMS]
        den += np.sum(B ** 2)
        num += sum(np.sum(B[np.ix_(g, g)] ** 2) for g in GROUPS.values())
    return float(num / den)


def refine_scores(prims, cam_rows, proj_mode: int = 0, with_lambda: bool = False):
    import oracle
    prm = oracle.Params(eta=ETA, z_near=Z_NEAR, clamp_k=CLAMP_K, e_col=E_COL, e_opa=E_OPA, e_lngem=E_LNGEM,
                        proj_mode=proj_mode)
    planes = oracle_planes(prims)
    F = oracle.stats(planes, eta=prm.eta)
    lam = oracle.lam(F, prm)
    D = oracle.score(planes, cam_rows, lam, prm)[0]
    return (D, lam) if with_lambda else D


def study(n: int = 40, V: int = 8, seed: int = 0, neighbourhoods: int = 1, k_nn: int = 10) -> dict:
    prims = make_scene(n, seed)
    cam_rows, cams = make_cameras(V)
    caches = [ViewCache(prims, c) for c in cams]
    Q = removal_errors(prims, caches)
    D_cov, lam = refine_scores(prims, cam_rows, 0, with_lambda=True)
    D_depth = refine_scores(prims, cam_rows, 1)
    alpha = np.array([1.0 / (1.0 + math.exp(-p.logit)) for p in prims])
    out = {"n": n, "views": V, "seed": seed,
           "spearman_D_cov_vs_removal": float(spearmanr(D_cov, Q)[0]),
           "spearman_D_depth_vs_removal": float(spearmanr(D_depth, Q)[0]),
           "spearman_opacity_vs_removal": float(spearmanr(alpha, Q)[0])}
    # REFINE's per-group weight (the same ranking for every group: only the
    # constant lambda^k differs) against each group's exact diagonal weight
    w = refine_group_weight(prims, D_cov, lam)
    W = exact_group_weights(prims, caches)
    for k in ("gem", "col", "opa"):
        out[f"spearman_w_vs_exact_diag_{k}"] = float(spearmanr(w, W[k])[0])
    # DER over k-nearest-neighbour sets (dense local regions)
    rng = np.random.default_rng(seed + 1)
    mus = np.stack([p.mu for p in prims])
    ders_p, ders_a, ident = [], [], []
    for _ in range(neighbourhoods):
        c = int(rng.integers(n))
        subset = list(np.argsort(np.sum((mus - mus[c]) ** 2, axis=1))[:k_nn + 1])
        J = jacobian(prims, caches, subset)
        H = gauss_newton(J)
        ders_p.append(der_primitives(H, len(subset)))
        ders_a.append(der_attributes(H, len(subset)))
        # removal = -alpha dR/dalpha exactly; dR/dlogit = alpha (1 - alpha) dR/dalpha
        for a, i in enumerate(subset):
            w_logit = H[a * N_PARAMS + 9, a * N_PARAMS + 9]
            al = alpha[i]
            ident.append((al ** 2 * w_logit / (al * (1 - al)) ** 2, Q[i]))
    out["der_primitives"] = float(np.mean(ders_p))
    out["der_attributes"] = float(np.mean(ders_a))
    est = np.array([e for e, q in ident])
    q = np.array([q for e, q in ident])
    out["removal_identity_max_rel_err"] = float(np.max(np.abs(est - q) / np.maximum(q, 1e-12)))
    return out


if __name__ == "__main__":
    import sys
    results = [study(n=100, V=8, seed=s, neighbourhoods=2, k_nn=30) for s in range(int(sys.argv[1]) if len(sys.argv) > 1 else 3)]
    print(json.dumps(results, indent=1))
