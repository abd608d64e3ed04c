"""Gaussian smoothing of the learned redundancy weight, in float64.

Sec. 3.1 places a Gaussian filter layer (standard deviation 20, 121 taps) right
after the redundancy weight layer.  Reading taken where the paper is silent: the
filter is the separable 2D Gaussian over the (mu, s) grid of each view, with
mirror padding (the edge sample is not repeated: ... c b | a b c ... | x y | x w ...),
applied to M before the weight is used; view rows are not mixed.

Each 1D pass is written as an explicit n x n matrix built from the definition
    y[i] = sum_{t=-r..r} w_t x[mirror(i + t)],   w_t = exp(-t^2 / (2 sigma^2)) / sum,
so the transpose used by the backward pass is that matrix transposed.
Pinned by tests against scipy's gaussian_filter1d (mode "mirror"), which states
the same filter independently, and by row sums and separability.
"""
from __future__ import annotations

import numpy as np


def taps(sigma, radius):
    """Normalised Gaussian weights w_t for t = -radius..radius."""
    t = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-0.5 * (t / sigma) ** 2)
    return w / w.sum()


def mirror(m, n):
    """Index of sample m after mirror padding of a length-n axis (needs |overhang| < n)."""
    if m < 0:
        return -m
    if m > n - 1:
        return 2 * (n - 1) - m
    return m


def pass_matrix(n, sigma, radius):
    """The n x n matrix of one 1D smoothing pass along an axis of length n."""
    if radius >= n:
        raise ValueError("radius must be below the axis length for mirror padding")
    w = taps(sigma, radius)
    S = np.zeros((n, n))
    for i in range(n):
        for t in range(-radius, radius + 1):
            S[i, mirror(i + t, n)] += w[t + radius]
    return S


def smooth_weights(M, sigma, radius):
    """M [V][n_theta][n_s] -> the smoothed weight, 1D passes along mu and along s."""
    M = np.asarray(M, np.float64)
    Smu = pass_matrix(M.shape[1], sigma, radius)
    Ss = pass_matrix(M.shape[2], sigma, radius)
    return np.matmul(np.matmul(Smu, M), Ss.T)


def smooth_weights_adjoint(G, sigma, radius):
    """Transpose of ``smooth_weights``: the same passes with the matrices transposed."""
    G = np.asarray(G, np.float64)
    Smu = pass_matrix(G.shape[1], sigma, radius)
    Ss = pass_matrix(G.shape[2], sigma, radius)
    return np.matmul(np.matmul(Smu.T, G), Ss)
