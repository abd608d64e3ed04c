"""Siddon's ray-driven projector (R. L. Siddon, Med. Phys. 12(2), 1985), float64.

Each ray from the source to a detector pixel centre is parameterised as
p(alpha) = p0 + alpha (p1 - p0), alpha in [0, 1].  The parameter values where it
crosses the voxel-boundary planes of each axis are merged and sorted; between
two consecutive crossings the ray lies in a single voxel (found from the
midpoint), and contributes (segment length) x (voxel value).  This gives the
exact line integral of the piecewise-constant voxel function, a different
discretisation from the bilinear cone-beam backprojector, so data made with it
does not share the reconstruction's own model.

Used by the tests to make projection data from voxelised phantoms and pinned
by exact chord lengths through boxes and single voxels.
"""
from __future__ import annotations

import numpy as np


def _planes(n, d, o):
    return (np.arange(n + 1) - n / 2.0) * d + o


def project_rays(vol, grid, p0, p1):
    """Line integrals of vol[nz][ny][nx] along segments p0[B,3] -> p1[B,3]."""
    p0 = np.atleast_2d(np.asarray(p0, np.float64))
    p1 = np.atleast_2d(np.asarray(p1, np.float64))
    B = p0.shape[0]
    d = p1 - p0
    length = np.linalg.norm(d, axis=1)
    planes = [_planes(grid.nx, grid.vx, grid.ox), _planes(grid.ny, grid.vy, grid.oy),
              _planes(grid.nz, grid.vz, grid.oz)]
    lo = np.zeros(B)
    hi = np.ones(B)
    cross = []
    with np.errstate(divide="ignore", invalid="ignore"):
        for ax in range(3):
            pl = planes[ax]
            a = (pl[None, :] - p0[:, ax:ax + 1]) / d[:, ax:ax + 1]
            par = d[:, ax] == 0.0
            a_first = np.where(par, -np.inf, np.minimum(a[:, 0], a[:, -1]))
            a_last = np.where(par, np.inf, np.maximum(a[:, 0], a[:, -1]))
            # a ray parallel to this axis misses the box unless it lies between the planes
            outside = par & ((p0[:, ax] < pl[0]) | (p0[:, ax] > pl[-1]))
            lo = np.maximum(lo, a_first)
            hi = np.minimum(hi, np.where(outside, -np.inf, a_last))
            cross.append(np.where(par[:, None], np.nan, a))
    al = np.concatenate(cross + [lo[:, None], hi[:, None]], axis=1)
    al = np.where((al >= lo[:, None]) & (al <= hi[:, None]), al, np.nan)
    al = np.sort(al, axis=1)              # NaNs sort to the end
    seg = np.diff(al, axis=1)
    mid = 0.5 * (al[:, 1:] + al[:, :-1])
    ok = np.isfinite(seg) & (seg > 0)
    mid = np.where(ok, mid, 0.0)
    pts = p0[:, None, :] + mid[..., None] * d[:, None, :]
    idx = []
    for ax, (n, dd, o) in enumerate(((grid.nx, grid.vx, grid.ox), (grid.ny, grid.vy, grid.oy),
                                     (grid.nz, grid.vz, grid.oz))):
        i = np.floor((pts[..., ax] - o) / dd + n / 2.0).astype(np.int64)
        ok &= (i >= 0) & (i < n)
        idx.append(np.clip(i, 0, n - 1))
    vals = vol[idx[2], idx[1], idx[0]]
    return np.sum(np.where(ok, seg * vals, 0.0), axis=1) * length


def project(vol, grid, views, view_ids=None):
    """Cone-beam projections g[V][nv][nu] of a voxel volume, one ray per pixel centre."""
    ids = range(len(views)) if view_ids is None else view_ids
    xs = (np.arange(grid.nu) - (grid.nu - 1) / 2.0) * grid.du
    ys = (np.arange(grid.nv) - (grid.nv - 1) / 2.0) * grid.dv
    out = []
    for v in ids:
        P = (views.det_center[v][None, None, :] + xs[None, :, None] * views.ex[v]
             + ys[:, None, None] * views.ey[v]).reshape(-1, 3)
        src = np.broadcast_to(views.src[v], P.shape)
        out.append(project_rays(vol, grid, src, P).reshape(grid.nv, grid.nu))
    return np.stack(out)
