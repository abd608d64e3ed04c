"""Structural similarity of two volumes and its gradient, in float64.

Eq. 13 adds an SSIM term to the MSE loss.  The paper does not spell SSIM out;
the reading taken is the standard definition (Wang et al., 2004) in 3D:
  mu_x = G * x, mu_y = G * y, s_xx = G * x^2 - mu_x^2, s_yy = G * y^2 - mu_y^2,
  s_xy = G * (x y) - mu_x mu_y,
  S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_xx + s_yy + C2)),
  SSIM = mean of S over the positions where the whole window lies in the volume,
with G the normalised Gaussian window of standard deviation 1.5 and radius 5
(11 taps per axis), C1 = (0.01 L)^2, C2 = (0.03 L)^2 and L the data range.

``window_moments`` forms the five window moments by explicit 11^3 sums;
``window_moments_separable`` by three 1D passes.  The gradient w.r.t. x is the
chain rule through the moments written out (``ssim_grad``); pinned by finite
differences.
"""
from __future__ import annotations

import numpy as np

SIGMA_W = 1.5
RADIUS_W = 5
K1, K2 = 0.01, 0.03


def window(sigma=SIGMA_W, radius=RADIUS_W):
    t = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-0.5 * (t / sigma) ** 2)
    return w / w.sum()


def window_moments(x, y, sigma=SIGMA_W, radius=RADIUS_W):
    """(mu_x, mu_y, E[x^2], E[y^2], E[xy]) on the valid grid, by explicit 3D window sums."""
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    w = window(sigma, radius)
    W3 = w[:, None, None] * w[None, :, None] * w[None, None, :]
    n = 2 * radius + 1
    out_shape = tuple(s - 2 * radius for s in x.shape)
    fields = [x, y, x * x, y * y, x * y]
    res = [np.zeros(out_shape) for _ in fields]
    for a in range(n):
        for b in range(n):
            for c in range(n):
                sl = (slice(a, a + out_shape[0]), slice(b, b + out_shape[1]), slice(c, c + out_shape[2]))
                for r, f in zip(res, fields):
                    r += W3[a, b, c] * f[sl]
    return res


def window_moments_separable(x, y, sigma=SIGMA_W, radius=RADIUS_W):
    """The same moments by three 1D valid convolutions (z, then y, then x)."""
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    w = window(sigma, radius)

    def conv(f, axis):
        n = f.shape[axis] - 2 * radius
        acc = 0.0
        for t in range(2 * radius + 1):
            acc = acc + w[t] * np.take(f, np.arange(t, t + n), axis=axis)
        return acc

    return [conv(conv(conv(f, 0), 1), 2) for f in (x, y, x * x, y * y, x * y)]


def ssim_map(x, y, data_range, sigma=SIGMA_W, radius=RADIUS_W, moments=window_moments):
    C1, C2 = (K1 * data_range) ** 2, (K2 * data_range) ** 2
    mx, my, exx, eyy, exy = moments(x, y, sigma, radius)
    A1, A2 = 2 * mx * my + C1, 2 * (exy - mx * my) + C2
    B1, B2 = mx * mx + my * my + C1, (exx - mx * mx) + (eyy - my * my) + C2
    return A1 * A2 / (B1 * B2)


def ssim(x, y, data_range, **kw):
    return float(np.mean(ssim_map(x, y, data_range, **kw)))


def ssim_grad(x, y, data_range, sigma=SIGMA_W, radius=RADIUS_W):
    """d SSIM / d x (y fixed), same shape as x.

    With S = A1 A2 / (B1 B2) as in ``ssim_map``, the derivatives of S at each
    valid position with respect to mu_x, E[x^2] and E[xy] are
      dS/dmu_x  = 2 mu_y (A2 - A1) / (B1 B2) - 2 mu_x S (1/B1 - 1/B2),
      dS/dE[x2] = -S / B2,        dS/dE[xy] = 2 A1 / (B1 B2),
    and each moment is G * (x, x^2, x y), so
      dSSIM/dx = (G^T dS/dmu_x + 2 x G^T dS/dE[x2] + y G^T dS/dE[xy]) / N,
    where G^T spreads a valid-grid field back over the window (zero outside)."""
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    C1, C2 = (K1 * data_range) ** 2, (K2 * data_range) ** 2
    mx, my, exx, eyy, exy = window_moments(x, y, sigma, radius)
    A1, A2 = 2 * mx * my + C1, 2 * (exy - mx * my) + C2
    B1, B2 = mx * mx + my * my + C1, (exx - mx * mx) + (eyy - my * my) + C2
    S = A1 * A2 / (B1 * B2)
    d_mu = 2 * my * (A2 - A1) / (B1 * B2) - 2 * mx * S * (1 / B1 - 1 / B2)
    d_exx = -S / B2
    d_exy = 2 * A1 / (B1 * B2)
    N = S.size
    w = window(sigma, radius)
    W3 = w[:, None, None] * w[None, :, None] * w[None, None, :]
    n = 2 * radius + 1
    spread = [np.zeros(x.shape) for _ in range(3)]
    for a in range(n):
        for b in range(n):
            for c in range(n):
                sl = (slice(a, a + S.shape[0]), slice(b, b + S.shape[1]), slice(c, c + S.shape[2]))
                for sp, d in zip(spread, (d_mu, d_exx, d_exy)):
                    sp[sl] += W3[a, b, c] * d
    return (spread[0] + 2 * x * spread[1] + y * spread[2]) / N
