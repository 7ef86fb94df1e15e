"""Seeded synthetic 3DGS scenes and camera rigs.

This module only draws inputs: it holds none of the scoring method's
arithmetic, so both the GPU path and the CPU oracle can consume its output.

Scene storage (the layout every entry point of the library reads) is
attribute-major ("SoA"): a float32 array ``planes[59][stride]`` where plane

    0..2    centre x, y, z (world units)
    3..5    log-scale of the three principal axes
    6..9    rotation quaternion, w first (w, x, y, z); not necessarily unit
    10      opacity logit
    11..13  SH degree-0 ("DC") coefficient for R, G, B
    14..58  the 45 higher-order SH coefficients (15 per channel)

i.e. the 59 parameters per primitive of the scene definition in Sec. 3.1,
Eq. (1) of the paper.

Camera rigs are float32 arrays ``cams[V][18]``: the world-to-camera rotation
R (9, row-major), translation t (3) so that p_cam = R p_world + t, then fx,
fy, cx, cy (pixels; Eq. (13)), image width W and height H (pixels).  Camera
axes follow the usual computer-vision convention: x right, y down, z forward.

Workloads (distributions chosen to resemble trained scenes of the sizes the
paper evaluates on, Sec. 4.1 and Table 2; no dataset content is used):

* ``small``  50k primitives, 16 ring cameras, 320x240, f=300
* ``medium`` 3M primitives in a [-20,20]^3 box, 200 hemisphere cameras,
  1237x822, f=1100
* ``large``  6M primitives, 64 clusters + 40% background, 300 cameras on a
  smooth closed trajectory, 1600x1060, f=1400
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

N_PLANES = 59
PLANE_XYZ = 0
PLANE_LOG_SCALE = 3
PLANE_QUAT = 6
PLANE_OPACITY = 10
PLANE_SH_DC = 11
PLANE_SH_REST = 14
CAM_FIELDS = 18
CAM_R, CAM_T, CAM_FX, CAM_FY, CAM_CX, CAM_CY, CAM_W, CAM_H = 0, 9, 12, 13, 14, 15, 16, 17


@dataclasses.dataclass(frozen=True)
class SceneSpec:
    """Recipe of one synthetic scene + camera rig."""

    name: str
    n: int
    n_clusters: int
    cluster_frac: float
    cluster_sigma: float
    center_half: float        # cluster centres ~ U[-center_half, center_half]^3
    uniform_half: float       # background ~ U[-uniform_half, uniform_half]^3
    rig: str                  # "ring" | "hemisphere" | "trajectory"
    n_views: int
    width: int
    height: int
    focal: float
    ratios: tuple
    seed: int

    def with_n(self, n: int, n_views: int | None = None) -> "SceneSpec":
        return dataclasses.replace(self, n=int(n),
                                   n_views=self.n_views if n_views is None else int(n_views))


SMALL = SceneSpec("small-50k-x16", 50_000, 8, 0.7, 0.5, 3.0, 5.0, "ring", 16,
                  320, 240, 300.0, (0.5,), 1000)
MEDIUM = SceneSpec("medium-3M-x200", 3_000_000, 8, 0.7, 2.0, 12.0, 20.0, "hemisphere", 200,
                   1237, 822, 1100.0, (0.5, 0.9), 1001)
LARGE = SceneSpec("large-6M-x300", 6_000_000, 64, 0.6, 2.0, 12.0, 20.0, "trajectory", 300,
                  1600, 1060, 1400.0, (0.66,), 1002)
SPECS = {"small": SMALL, "medium": MEDIUM, "large": LARGE}


def make_planes(spec: SceneSpec, stride: int | None = None, rng=None) -> np.ndarray:
    """Draw ``spec.n`` primitives into a float32 ``[59][stride]`` array.

    Per primitive: centre from one of ``n_clusters`` isotropic Gaussian
    clusters (fraction ``cluster_frac``) or uniform in a box; log-scales
    i.i.d. N(-4.5, 1); quaternion a normalised N(0, I4) draw; opacity logit
    N(0, 1.5); SH DC N(0, 0.5); higher SH N(0, 0.05) (all std devs).
    Padding columns beyond ``n`` are zero.
    """
    n = int(spec.n)
    stride = n if stride is None else int(stride)
    if stride < n:
        raise ValueError("stride < n")
    if rng is None:
        rng = np.random.default_rng(spec.seed)
    out = np.zeros((N_PLANES, stride), dtype=np.float32)
    if n == 0:
        return out
    n_cl = int(round(spec.cluster_frac * n))
    centres = rng.uniform(-spec.center_half, spec.center_half, size=(spec.n_clusters, 3))
    which = rng.integers(0, spec.n_clusters, size=n_cl)
    xyz = np.empty((n, 3))
    xyz[:n_cl] = centres[which] + rng.normal(0.0, spec.cluster_sigma, size=(n_cl, 3))
    xyz[n_cl:] = rng.uniform(-spec.uniform_half, spec.uniform_half, size=(n - n_cl, 3))
    xyz = xyz[rng.permutation(n)]          # interleave clusters and background
    out[0:3, :n] = xyz.T
    out[3:6, :n] = rng.normal(-4.5, 1.0, size=(3, n))
    q = rng.normal(0.0, 1.0, size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    out[6:10, :n] = q
    out[10, :n] = rng.normal(0.0, 1.5, size=n)
    out[11:14, :n] = rng.normal(0.0, 0.5, size=(3, n))
    out[14:59, :n] = rng.normal(0.0, 0.05, size=(45, n))
    return out


def look_at(eye, target, up=(0.0, 0.0, 1.0)):
    """World-to-camera (R, t) for a camera at ``eye`` looking at ``target``.

    Rows of R are the camera's right, down and forward axes in world
    coordinates; t = -R eye.
    """
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up = np.asarray(up, dtype=np.float64)
    if abs(float(np.dot(fwd, up))) > 0.99:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    return R, -R @ eye


def pack_camera(R, t, fx, fy, cx, cy, W, H) -> np.ndarray:
    row = np.empty(CAM_FIELDS, dtype=np.float64)
    row[0:9] = np.asarray(R, dtype=np.float64).reshape(9)
    row[9:12] = t
    row[12:18] = (fx, fy, cx, cy, W, H)
    return row.astype(np.float32)


def make_cameras(spec: SceneSpec, rng=None) -> np.ndarray:
    """Camera rig of ``spec`` as float32 ``[V][18]``."""
    if rng is None:
        rng = np.random.default_rng(spec.seed + 7919)
    V = int(spec.n_views)
    W, H, f = spec.width, spec.height, spec.focal
    cx, cy = W / 2.0, H / 2.0
    rows = []
    if spec.rig == "ring":
        for j in range(V):
            a = 2.0 * math.pi * j / V
            eye = (8.0 * math.cos(a), 8.0 * math.sin(a), 0.0)
            R, t = look_at(eye, (0.0, 0.0, 0.0))
            rows.append(pack_camera(R, t, f, f, cx, cy, W, H))
    elif spec.rig == "hemisphere":
        golden = math.pi * (3.0 - math.sqrt(5.0))
        for j in range(V):
            zc = (j + 0.5) / V
            elev = math.asin(zc) + math.radians(rng.uniform(-5.0, 5.0))
            elev = min(max(elev, 0.0), math.radians(89.0))
            azim = j * golden + math.radians(rng.uniform(-5.0, 5.0))
            rad = rng.uniform(4.0, 6.0)
            eye = (rad * math.cos(elev) * math.cos(azim), rad * math.cos(elev) * math.sin(azim),
                   rad * math.sin(elev))
            R, t = look_at(eye, (0.0, 0.0, 0.0))
            rows.append(pack_camera(R, t, f, f, cx, cy, W, H))
    elif spec.rig == "trajectory":
        amp = rng.normal(0.0, 1.0, size=(4, 3))
        ph = rng.uniform(0.0, 2.0 * math.pi, size=(4, 3))
        th = 2.0 * math.pi * np.arange(V) / V

        def fourier(k):
            return sum(amp[k, h] * np.cos((h + 1) * th + ph[k, h]) for h in range(3))

        def rescale(x, lo, hi):
            span = x.max() - x.min()
            return lo + (hi - lo) * (x - x.min()) / (span if span > 0 else 1.0)

        rad = rescale(fourier(0), 6.0, 10.0)
        hgt = rescale(fourier(1), 1.0, 4.0)
        tx = 0.5 * fourier(2) / (np.abs(fourier(2)).max() + 1e-12)
        ty = 0.5 * fourier(3) / (np.abs(fourier(3)).max() + 1e-12)
        for j in range(V):
            eye = (rad[j] * math.cos(th[j]), rad[j] * math.sin(th[j]), hgt[j])
            R, t = look_at(eye, (tx[j], ty[j], 0.0))
            rows.append(pack_camera(R, t, f, f, cx, cy, W, H))
    else:
        raise ValueError(f"unknown rig {spec.rig!r}")
    if not rows:
        return np.zeros((0, CAM_FIELDS), dtype=np.float32)
    return np.stack(rows).astype(np.float32)



# ------------------------------------------------------------ 2-byte storage
#
# Two 2-byte scene formats.  Mixed: planes 0..10 (centre, log-scale,
# quaternion, opacity) as bfloat16 and planes 11..58 (SH coefficients) as IEEE
# half, held as int16 bit patterns in the same [59][stride] layout.  Half:
# every plane IEEE half (float16 arrays); its 11-bit significand keeps
# centres 8 times closer to their FP32 values than bfloat16's 8 bits.
# Conversion from float32 rounds to nearest, ties to even, on the host.

N_GEOM_PLANES = 11


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (uint16), round to nearest even; NaN
    stays a quiet NaN of the same sign, overflow rounds to infinity."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    rounded = (u.astype(np.uint64) + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = rounded.astype(np.uint16)
    nan = np.isnan(np.asarray(x, dtype=np.float32))
    out[nan] = ((u[nan] >> 16) | 0x0040).astype(np.uint16)
    return out


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def quantize_bf16_f16(planes: np.ndarray) -> np.ndarray:
    """float32 planes [59][stride] -> int16 bit patterns of the mixed format."""
    planes = np.asarray(planes, dtype=np.float32)
    out = np.empty(planes.shape, dtype=np.uint16)
    out[:N_GEOM_PLANES] = f32_to_bf16_bits(planes[:N_GEOM_PLANES])
    out[N_GEOM_PLANES:] = planes[N_GEOM_PLANES:].astype(np.float16).view(np.uint16)
    return out.view(np.int16)


def quantize_f16(planes: np.ndarray) -> np.ndarray:
    """float32 planes [59][stride] -> the half 2-byte format: every plane IEEE
    half, round to nearest even (numpy's conversion).  Values beyond the half
    range (|x| > 65504) become infinities, which the library counts as
    non-finite inputs."""
    with np.errstate(over="ignore"):
        return np.asarray(planes, dtype=np.float32).astype(np.float16)


def dequantize_f16(planes: np.ndarray) -> np.ndarray:
    return np.asarray(planes, dtype=np.float16).astype(np.float32)


def dequantize_bf16_f16(bits: np.ndarray) -> np.ndarray:
    """int16 bit patterns of the mixed format -> float32 (exact)."""
    u = np.asarray(bits).view(np.uint16)
    out = np.empty(u.shape, dtype=np.float32)
    out[:N_GEOM_PLANES] = bf16_bits_to_f32(u[:N_GEOM_PLANES])
    out[N_GEOM_PLANES:] = u[N_GEOM_PLANES:].view(np.float16).astype(np.float32)
    return out


# ------------------------------------------------------------------ serving
#
# The serving workload: prune jobs on resident scenes drawn like the small
# scene (clusters in [-3,3]^3 with sigma 0.5, background in [-5,5]^3, ring
# cameras at radius 8, 320x240, f = 300) with a primitive count log-uniform
# in [0.2M, 6M]; each job brings 50..300 ring cameras and a prune ratio
# uniform in [0.3, 0.9]; jobs arrive as a Poisson process (20 per second).

SERVE_N_RANGE = (200_000, 6_000_000)
SERVE_VIEWS_RANGE = (50, 300)
SERVE_RATIO_RANGE = (0.3, 0.9)
SERVE_RATE = 20.0


def serve_scene_specs(count: int, seed: int = 3000, n_range=SERVE_N_RANGE) -> list:
    """Specs of `count` resident scenes whose primitive counts are evenly
    spaced in log over n_range, both ends included (so the largest scene of
    the law, which sets the tail latency, is served), and jobs that pick a
    scene uniformly see a discretised log-uniform law."""
    lo, hi = np.log(n_range[0]), np.log(n_range[1])
    ns = np.round(np.exp(lo + np.arange(count) / max(count - 1, 1) * (hi - lo))).astype(np.int64)
    return [dataclasses.replace(SMALL, name=f"serve-{j}-{int(n)}", n=int(n), seed=seed + 1 + j)
            for j, n in enumerate(ns)]


def serve_requests(count: int, n_scenes: int, seed: int = 3100, rate: float = SERVE_RATE,
                   views_range=SERVE_VIEWS_RANGE, ratio_range=SERVE_RATIO_RANGE):
    """(arrival seconds, [(scene index, views, ratio)]) of `count` jobs."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count))
    jobs = [(int(rng.integers(0, n_scenes)), int(rng.integers(views_range[0], views_range[1] + 1)),
             float(rng.uniform(*ratio_range))) for _ in range(count)]
    return arrivals, jobs


def ring_cameras(n_views: int) -> np.ndarray:
    """The small scene's ring rig with n_views cameras."""
    return make_cameras(SMALL.with_n(SMALL.n, n_views=n_views))
