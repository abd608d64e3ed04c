"""Random-ellipsoid phantoms, their exact cone-beam line integrals, noise.

Phantom recipe (stands in for the paper's simulated training objects, Sec. 3.3,
and for its clinical test data, which is not used): K ellipsoids with
semi-axes U[2, 12] mm, centres uniform in a ball of radius max(0, L/2 - 12 mm)
about the isocentre (L = smallest volume side), uniformly random orientation,
densities U[0.1, 1.0]; overlapping ellipsoids add.  Projections are exact chord
lengths times density along each source-to-pixel-centre ray (no voxelisation),
so GPU reconstructions are never fed data made by their own discretisation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

MU_WATER_PER_MM = 0.02   # attenuation per unit density, used only by the noise model


@dataclass
class Ellipsoids:
    centers: np.ndarray    # [K, 3] mm
    axes: np.ndarray       # [K, 3] semi-axes, mm
    rot: np.ndarray        # [K, 3, 3] columns = ellipsoid axes in world frame
    density: np.ndarray    # [K]


def _rand_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def random_ellipsoids(n, side_mm, seed, axis_range=(2.0, 12.0), dens_range=(0.1, 1.0)):
    rng = np.random.Generator(np.random.PCG64(seed))
    rad = max(0.0, side_mm / 2 - axis_range[1])
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rad * rng.uniform(0, 1, n) ** (1.0 / 3.0)
    centers = d * r[:, None]
    axes = rng.uniform(axis_range[0], axis_range[1], size=(n, 3))
    rot = np.stack([_rand_rotation(rng) for _ in range(n)])
    dens = rng.uniform(dens_range[0], dens_range[1], n)
    return Ellipsoids(centers, axes, rot, dens)


def ball(center, radius, density=1.0):
    return Ellipsoids(np.asarray([center], np.float64), np.full((1, 3), float(radius)),
                      np.eye(3)[None].copy(), np.asarray([density], np.float64))


def voxel_centers(grid):
    xs = (np.arange(grid.nx) - (grid.nx - 1) / 2) * grid.vx + grid.ox
    ys = (np.arange(grid.ny) - (grid.ny - 1) / 2) * grid.vy + grid.oy
    zs = (np.arange(grid.nz) - (grid.nz - 1) / 2) * grid.vz + grid.oz
    return xs, ys, zs


def voxelize(ell: Ellipsoids, grid) -> np.ndarray:
    """Point-sampled density at voxel centres, array [nz][ny][nx] float64."""
    xs, ys, zs = voxel_centers(grid)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1)
    out = np.zeros(X.shape)
    for c, a, R, rho in zip(ell.centers, ell.axes, ell.rot, ell.density):
        u = (P - c) @ R / a
        out += rho * (np.einsum("...i,...i->...", u, u) <= 1.0)
    return out


def project_ellipsoids(ell: Ellipsoids, grid, views, device="cpu", dtype=torch.float64,
                       view_chunk=32):
    """Exact line integrals g[V][nv][nu] through the ellipsoids along the rays
    from each source to each detector pixel centre (torch, float64 math)."""
    dev = torch.device(device)
    V = len(views)
    xs = (torch.arange(grid.nu, dtype=torch.float64, device=dev) - (grid.nu - 1) / 2) * grid.du
    ys = (torch.arange(grid.nv, dtype=torch.float64, device=dev) - (grid.nv - 1) / 2) * grid.dv
    out = torch.empty((V, grid.nv, grid.nu), dtype=dtype, device=dev)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    C, A, R, rho = t(ell.centers), t(ell.axes), t(ell.rot), t(ell.density)
    for v0 in range(0, V, view_chunk):
        v1 = min(V, v0 + view_chunk)
        src = t(views.src[v0:v1])[:, None, None, :]
        O = t(views.det_center[v0:v1])[:, None, None, :]
        ex = t(views.ex[v0:v1])[:, None, None, :]
        ey = t(views.ey[v0:v1])[:, None, None, :]
        P = O + xs[None, None, :, None] * ex + ys[None, :, None, None] * ey
        d = P - src
        d = d / torch.linalg.norm(d, dim=-1, keepdim=True)
        acc = torch.zeros(d.shape[:-1], dtype=torch.float64, device=dev)
        for k in range(C.shape[0]):
            q = ((src - C[k]) @ R[k]) / A[k]
            dd = (d @ R[k]) / A[k]
            al = (dd * dd).sum(-1)
            be = (dd * q).sum(-1)
            ga = (q * q).sum(-1)
            disc = be * be - al * (ga - 1.0)
            acc += rho[k] * 2.0 * torch.sqrt(torch.clamp(disc, min=0.0)) / al
        out[v0:v1] = acc.to(dtype)
    return out


def add_poisson_noise(g: torch.Tensor, photons: float, seed: int, mu=MU_WATER_PER_MM):
    """Poisson counts at I0 = photons per ray on attenuation mu*g; returns the
    log-converted noisy line integral in the units of g."""
    gen = torch.Generator(device=g.device)
    gen.manual_seed(seed)
    lam = photons * torch.exp(-mu * g.to(torch.float64))
    n = torch.poisson(lam, generator=gen)
    return (-torch.log(torch.clamp(n, min=1.0) / photons) / mu).to(g.dtype)


def rand_array(shape, seed, lo=-1.0, hi=1.0, dtype=np.float32):
    """Uniform random array (numpy, PCG64), values rounded to dtype."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=shape).astype(dtype)


def gaussian_blobs(n, side_mm, seed, sigma_range=(2.0, 5.0)):
    """Isotropic Gaussian blobs (smooth phantom): centres [K,3], sigmas [K], amplitudes [K]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rad = max(0.0, side_mm / 2 - 2.5 * sigma_range[1])
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    c = d * (rad * rng.uniform(0, 1, n) ** (1 / 3))[:, None]
    return c, rng.uniform(*sigma_range, n), rng.uniform(0.5, 1.0, n)


def project_gaussian_blobs(blobs, grid, views):
    """Exact line integrals (float64 numpy) of a sum of isotropic Gaussians
    A exp(-|p-c|^2 / (2 s^2)) along source-to-pixel rays: A s sqrt(2 pi) exp(-d^2/(2 s^2)),
    d = distance from the centre to the ray."""
    C, S, A = blobs
    xs = (np.arange(grid.nu) - (grid.nu - 1) / 2) * grid.du
    ys = (np.arange(grid.nv) - (grid.nv - 1) / 2) * grid.dv
    out = np.zeros((len(views), grid.nv, grid.nu))
    for v in range(len(views)):
        P = (views.det_center[v] + xs[None, :, None] * views.ex[v] + ys[:, None, None] * views.ey[v])
        d = P - views.src[v]
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        for c, s, a in zip(C, S, A):
            q = c - views.src[v]
            along = (q * d).sum(-1)
            dist2 = (q * q).sum() - along ** 2
            out[v] += a * s * math.sqrt(2 * math.pi) * np.exp(-np.maximum(dist2, 0) / (2 * s * s))
    return out


def voxelize_gaussian_blobs(blobs, grid):
    C, S, A = blobs
    xs, ys, zs = voxel_centers(grid)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    out = np.zeros(X.shape)
    for c, s, a in zip(C, S, A):
        out += a * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2 * s * s))
    return out


def voxelize_torch(ell: Ellipsoids, grid, device="cpu", dtype=torch.float32, z_chunk=16):
    """Same point-sampled phantom as ``voxelize`` computed with torch (for large volumes)."""
    dev = torch.device(device)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    xs = (torch.arange(grid.nx, dtype=torch.float64, device=dev) - (grid.nx - 1) / 2) * grid.vx + grid.ox
    ys = (torch.arange(grid.ny, dtype=torch.float64, device=dev) - (grid.ny - 1) / 2) * grid.vy + grid.oy
    zs = (torch.arange(grid.nz, dtype=torch.float64, device=dev) - (grid.nz - 1) / 2) * grid.vz + grid.oz
    out = torch.zeros((grid.nz, grid.ny, grid.nx), dtype=dtype, device=dev)
    C, A, R, rho = t(ell.centers), t(ell.axes), t(ell.rot), t(ell.density)
    for z0 in range(0, grid.nz, z_chunk):
        Z, Y, X = torch.meshgrid(zs[z0:z0 + z_chunk], ys, xs, indexing="ij")
        Pt = torch.stack([X, Y, Z], dim=-1)
        acc = torch.zeros(Z.shape, dtype=torch.float64, device=dev)
        for k in range(C.shape[0]):
            u = ((Pt - C[k]) @ R[k]) / A[k]
            acc += rho[k] * ((u * u).sum(-1) <= 1.0)
        out[z0:z0 + z_chunk] = acc.to(dtype)
    return out
