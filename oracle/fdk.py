"""Textbook Feldkamp-Davis-Kress reconstruction for a circular orbit, float64.

Written from the FDK formula as usually stated for a virtual detector through
the rotation axis (Feldkamp, Davis & Kress, JOSA A 1(6), 1984; Kak & Slaney,
"Principles of Computerized Tomographic Imaging", ch. 3):

    f(x) = 1/2 sum_beta dbeta (R^2 / U^2) Q_beta(p(x), zeta(x)),
    Q_beta = [ P_beta(p, zeta) R / sqrt(R^2 + p^2 + zeta^2) ] *_p h,

with R the source-isocentre distance, U the source-to-voxel depth along the
central ray, (p, zeta) the virtual-detector coordinates (physical detector
coordinates scaled by R/D) and h the Ram-Lak ramp kernel sampled at the virtual
pitch tau: h(0) = 1/(4 tau^2), h(n even) = 0, h(n odd) = -1/(n pi tau)^2.

It shares nothing with ``pipeline`` (different filter, different weights, its
own interpolation), which makes it an independent check of the Defrise-Clack
chain: for a circle with M = 1/2 the chain reduces to FDK in the continuum.
"""
from __future__ import annotations

import math

import numpy as np


def ramlak(n_taps, tau):
    n = np.arange(-(n_taps - 1), n_taps)
    h = np.zeros(n.shape)
    h[n == 0] = 1.0 / (4 * tau * tau)
    odd = (n % 2) != 0
    h[odd] = -1.0 / (n[odd] * math.pi * tau) ** 2
    return h


def fdk_circle(g, grid, views, points=None):
    """FDK of projections g[V][nv][nu] acquired on an equally spaced full circle."""
    V = len(views)
    R = float(np.linalg.norm(views.src[0]))
    D = float(np.linalg.norm(views.src[0] - views.det_center[0]))
    tau_p, tau_z = grid.du * R / D, grid.dv * R / D
    p = (np.arange(grid.nu) - (grid.nu - 1) / 2.0) * tau_p
    z = (np.arange(grid.nv) - (grid.nv - 1) / 2.0) * tau_z
    cw = R / np.sqrt(R * R + p[None, :] ** 2 + z[:, None] ** 2)
    h = ramlak(grid.nu, tau_p)
    if points is None:
        xs = (np.arange(grid.nx) - (grid.nx - 1) / 2.0) * grid.vx + grid.ox
        ys = (np.arange(grid.ny) - (grid.ny - 1) / 2.0) * grid.vy + grid.oy
        zs = (np.arange(grid.nz) - (grid.nz - 1) / 2.0) * grid.vz + grid.oz
        Zg, Yg, Xg = np.meshgrid(zs, ys, xs, indexing="ij")
        points = np.stack([Xg, Yg, Zg], axis=-1)
    X = np.asarray(points, np.float64)
    f = np.zeros(X.shape[:-1])
    dbeta = 2 * math.pi / V
    for v in range(V):
        a = views.src[v]
        e_src = a / R                     # unit vector isocentre -> source
        e_p = views.ex[v]
        e_z = views.ey[v]
        weighted = np.asarray(g[v], np.float64) * cw
        Q = np.stack([tau_p * np.convolve(row, h, mode="full")[grid.nu - 1: 2 * grid.nu - 1]
                      for row in weighted])
        U = R - X @ e_src                 # depth of the point from the source
        pp = R * (X @ e_p) / U
        zz = R * (X @ e_z) / U
        fi = pp / tau_p + (grid.nu - 1) / 2.0
        fj = zz / tau_z + (grid.nv - 1) / 2.0
        i0 = np.floor(fi).astype(int)
        j0 = np.floor(fj).astype(int)
        wi, wj = fi - i0, fj - j0
        val = np.zeros(X.shape[:-1])
        for dj, wy in ((0, 1 - wj), (1, wj)):
            for di, wx in ((0, 1 - wi), (1, wi)):
                ii, jj = i0 + di, j0 + dj
                ok = (ii >= 0) & (ii < grid.nu) & (jj >= 0) & (jj < grid.nv)
                val += np.where(ok, wx * wy * Q[np.clip(jj, 0, grid.nv - 1), np.clip(ii, 0, grid.nu - 1)], 0.0)
        f += 0.5 * dbeta * (R * R / (U * U)) * val
    return f
