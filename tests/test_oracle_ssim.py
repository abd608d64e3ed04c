"""Pins of the oracle's 3D SSIM (eq. 13's structural term) and its gradient."""
import numpy as np
import pytest

from oracle import ssim as Q


def vols(seed, shape=(14, 15, 13)):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0, 1, shape), rng.uniform(0, 1, shape)


def test_identical_volumes_score_one_and_the_score_is_symmetric():
    x, y = vols(1)
    assert abs(Q.ssim(x, x, 1.0) - 1.0) < 1e-14
    assert abs(Q.ssim(x, y, 1.0) - Q.ssim(y, x, 1.0)) < 1e-14
    assert Q.ssim(x, y, 1.0) < 0.5


def test_constant_volumes_closed_form():
    """For x = a and y = b everywhere the variances vanish: S = (2ab + C1)/(a^2 + b^2 + C1)."""
    a, b, L = 0.3, 0.7, 1.0
    C1 = (Q.K1 * L) ** 2
    x, y = np.full((12, 12, 12), a), np.full((12, 12, 12), b)
    # the variances cancel to ~1e-15 in float64, against C2 = 9e-4
    assert abs(Q.ssim(x, y, L) - (2 * a * b + C1) / (a * a + b * b + C1)) < 1e-11


def test_separable_moments_equal_explicit_window_sums():
    x, y = vols(2)
    for m1, m2 in zip(Q.window_moments(x, y), Q.window_moments_separable(x, y)):
        assert np.allclose(m1, m2, rtol=1e-12, atol=1e-14)
    w = Q.window()
    assert len(w) == 11 and abs(w.sum() - 1) < 1e-15 and abs(w[5] / w[6] - np.exp(0.5 / 1.5 ** 2)) < 1e-12


def test_gradient_matches_finite_differences():
    x, y = vols(3, (12, 13, 11))
    g = Q.ssim_grad(x, y, 1.0)
    rng = np.random.Generator(np.random.PCG64(4))
    for _ in range(6):
        idx = tuple(int(rng.integers(0, s)) for s in x.shape)
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (Q.ssim(xp, y, 1.0) - Q.ssim(xm, y, 1.0)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * max(1e-3, abs(g).max()), (idx, fd, g[idx])
    # a voxel that no valid window covers has zero gradient only if outside every window:
    # every voxel is inside some window here (radius 5 < half of each size), so none is zero
    assert np.count_nonzero(g) == g.size
