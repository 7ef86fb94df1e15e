"""The footprint bound the culling and the view loop's screen rely on, pinned
by brute force on the CPU (no GPU code runs here).

A primitive's 3-sigma footprint radius r (paper Eq. 14-16: the larger
eigenvalue of the projected covariance J R Sigma R^T J^T) obeys
r z <= 3 s_max |z J|_2, and over the clamp box |x/z| <= limx, |y/z| <= limy
the spectral norm |z J|_2 is largest at a corner of the box.  The kernels
compute that corner value in closed form; these tests restate the formula and
check it against dense sampling of the box and against random primitives.
"""
import numpy as np


def corner_spectral_norm(fx, fy, limx, limy):
    """Closed form of max |z J|_2 over the clamp box (its corner value)."""
    a = fx * fx * (1.0 + limx * limx)
    c = fy * fy * (1.0 + limy * limy)
    b = fx * fy * limx * limy
    return np.sqrt(0.5 * (a + c) + np.sqrt(0.25 * (a - c) ** 2 + b * b))


def zj(fx, fy, xh, yh):
    return np.array([[fx, 0.0, -fx * xh], [0.0, fy, -fy * yh]])


def test_corner_value_dominates_the_clamp_box():
    rng = np.random.default_rng(3)
    for _ in range(200):
        fx, fy = rng.uniform(100.0, 3000.0, size=2)
        limx, limy = rng.uniform(0.05, 2.0, size=2)
        bound = corner_spectral_norm(fx, fy, limx, limy)
        xs = np.linspace(-limx, limx, 41)
        ys = np.linspace(-limy, limy, 41)
        best = max(np.linalg.norm(zj(fx, fy, x, y), 2) for x in xs for y in ys)
        # attained at a corner, and never exceeded inside the box
        assert best <= bound * (1.0 + 1e-12)
        assert best >= bound * (1.0 - 1e-12)


def test_corner_value_is_below_the_frobenius_bound():
    rng = np.random.default_rng(4)
    for _ in range(100):
        fx, fy = rng.uniform(100.0, 3000.0, size=2)
        limx, limy = rng.uniform(0.05, 2.0, size=2)
        frob = np.sqrt(fx * fx * (1.0 + limx * limx) + fy * fy * (1.0 + limy * limy))
        spec = corner_spectral_norm(fx, fy, limx, limy)
        assert spec <= frob * (1.0 + 1e-12)
        assert spec >= frob / np.sqrt(2.0) * (1.0 - 1e-12)


def test_footprint_radius_never_exceeds_the_bound():
    """r z = 3 sqrt(lambda_max(zJ R L L^T R^T (zJ)^T)) <= 3 s_max corner norm
    for random rotations, scales, view rotations and clamped positions."""
    rng = np.random.default_rng(5)

    def rot(q):
        w, x, y, z = q / np.linalg.norm(q)
        return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                         [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                         [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])

    worst = 0.0
    for _ in range(2000):
        fx, fy = rng.uniform(100.0, 3000.0, size=2)
        limx, limy = rng.uniform(0.05, 2.0, size=2)
        s = np.exp(rng.normal(-3.0, 1.5, size=3))
        L = rot(rng.normal(size=4)) * s[None, :]
        Rv = rot(rng.normal(size=4))
        xh, yh = rng.uniform(-limx, limx), rng.uniform(-limy, limy)
        A = zj(fx, fy, xh, yh) @ Rv @ L
        rz = 3.0 * np.sqrt(np.linalg.eigvalsh(A @ A.T).max())
        bound = 3.0 * s.max() * corner_spectral_norm(fx, fy, limx, limy)
        assert rz <= bound * (1.0 + 1e-12)
        worst = max(worst, rz / bound)
    assert worst > 0.5   # the bound is not vacuous
