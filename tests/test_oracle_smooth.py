"""Pins of the oracle's Gaussian weight smoothing (Sec. 3.1: sigma 20, 121 taps).

The oracle builds each 1D pass as an explicit matrix; these tests tie it to an
independent statement of the same filter (scipy.ndimage.gaussian_filter1d with
mirror padding), to hand-computed boundary cases of the mirror rule, to the
invariants of a normalised kernel, and to the adjoint identity.
"""
import numpy as np
import pytest

from oracle import smooth as S


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("sigma, radius, shape", [(20.0, 60, (2, 130, 151)), (3.0, 9, (3, 17, 23)),
                                                  (1.5, 4, (1, 6, 9))])
def test_matches_scipy_gaussian_filter_with_mirror_padding(sigma, radius, shape):
    from scipy.ndimage import gaussian_filter1d
    rng = np.random.Generator(np.random.PCG64(1))
    M = rng.uniform(-1, 0, shape)
    ref = gaussian_filter1d(M, sigma, axis=1, mode="mirror", truncate=radius / sigma)
    ref = gaussian_filter1d(ref, sigma, axis=2, mode="mirror", truncate=radius / sigma)
    assert rel(S.smooth_weights(M, sigma, radius), ref) < 1e-12


def test_mirror_boundary_by_hand():
    """n = 5, radius 2: a unit sample at index 0 spreads w0 w1 w2 inward; one at
    index 1 is met twice by the first output (from +1 and from the mirrored -1)."""
    w = S.taps(1.3, 2)
    w0, w1, w2 = w[2], w[3], w[4]
    Sm = S.pass_matrix(5, 1.3, 2)
    assert np.allclose(Sm[:, 0], [w0, w1, w2, 0, 0], atol=1e-15)
    assert np.allclose(Sm[:, 1], [2 * w1, w0 + w2, w1, w2, 0], atol=1e-15)


def test_taps_rows_and_interior_delta():
    w = S.taps(20.0, 60)
    assert len(w) == 121 and abs(w.sum() - 1) < 1e-15 and np.allclose(w, w[::-1], rtol=0, atol=0)
    assert abs(w[60] / w[80] - np.exp(0.5)) < 1e-12            # 20 samples = one sigma
    Sm = S.pass_matrix(200, 20.0, 60)
    assert np.allclose(Sm.sum(axis=1), 1.0, atol=1e-14)        # constants are preserved
    d = np.zeros((1, 200, 200))
    d[0, 90, 110] = 1.0
    assert np.allclose(S.smooth_weights(d, 20.0, 60)[0, 90 - 60:90 + 61, 110 - 60:110 + 61], np.outer(w, w),
                       atol=1e-16)


def test_adjoint_identity():
    rng = np.random.Generator(np.random.PCG64(2))
    x, y = rng.normal(size=(2, 37, 41)), rng.normal(size=(2, 37, 41))
    lhs = float(np.sum(S.smooth_weights(x, 4.0, 12) * y))
    rhs = float(np.sum(x * S.smooth_weights_adjoint(y, 4.0, 12)))
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(x) * np.linalg.norm(y)


def test_radius_must_fit_the_axis():
    with pytest.raises(ValueError):
        S.pass_matrix(10, 2.0, 10)
