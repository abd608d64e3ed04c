"""The discretised reconstruction of eq. 12, stage by stage, in float64.

    f = A3d^T w_d A2d^T D w_red w_sino D A2d w_cos g            (eq. 12)

Discretisation (the readings taken where the paper is silent):
  * detector pixel (i, j) sits at x_i = (i - (nu-1)/2) du, y_j = (j - (nv-1)/2) dv
    in the detector frame (origin at the detector centre, Fig. 1);
  * Radon grid: mu_k = k pi / n_theta, k = 0..n_theta-1 (angular range pi,
    Table 2), s_m = (m - (n_s-1)/2) ds;
  * A2d^T is pixel-driven linear interpolation of each sinogram row at
    s = x cos mu + y sin mu summed over mu with weight pi / n_theta (the
    integral over [0, pi) in eq. 8); A2d is its transpose scaled to a line
    integral, (du dv / ds) sum_p g_p Lambda((s_p - s_m) / ds), with the hat
    function Lambda(t) = max(0, 1 - |t|) and zero outside every array;
  * the derivative D = d/ds is the zero-padded central difference;
  * w_sino * w_red collapse (eqs. 7, 10 with theta = (D n_mu + s l_z)/sqrt(s^2+D^2))
    to  W = M * c_geo,  c_geo = -|D (t.n_mu) + s (t.l_z)| / (4 pi^2 D^2),
    where t = a'(lambda) dlambda carries the view quadrature weight;
  * the detector weight w_d = x^2+y^2+D^2 and the 1/|x-a|^2 of eq. 5 combine at
    the voxel's exact projection into D^2/U^2, U = (a - x).l_z (depth), which
    is what the cone-beam backprojection applies;  ``cone_bp_literal`` keeps the
    paper's order (w_d at pixel centres, then 1/|x-a|^2) for comparison.

Array layouts (row-major, last index fastest): projections g[V][nv][nu];
sinograms R, H, M[V][n_theta][n_s]; volume f[nz][ny][nx].
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI2 = 4.0 * math.pi * math.pi


# ----------------------------------------------------------------- geometry
def view_frame(views, v):
    """(a, O, l_x, l_y, l_z, D, t) of view v; D = (a - O).l_z (Fig. 1, eq. 6)."""
    a = np.asarray(views.src[v], np.float64)
    O = np.asarray(views.det_center[v], np.float64)
    lx = np.asarray(views.ex[v], np.float64)
    ly = np.asarray(views.ey[v], np.float64)
    lz = np.cross(lx, ly)
    D = float(np.dot(a - O, lz))
    return a, O, lx, ly, lz, D, np.asarray(views.tangent[v], np.float64)


def det_coords(grid):
    x = (np.arange(grid.nu) - (grid.nu - 1) / 2.0) * grid.du
    y = (np.arange(grid.nv) - (grid.nv - 1) / 2.0) * grid.dv
    return x, y


def radon_coords(grid):
    mu = np.arange(grid.n_theta) * (math.pi / grid.n_theta)
    s = (np.arange(grid.n_s) - (grid.n_s - 1) / 2.0) * grid.ds
    return mu, s


def hat(t):
    return np.maximum(0.0, 1.0 - np.abs(t))


# ----------------------------------------------------- O1: cosine weight
def w_cos(grid, D):
    """w_cos = D / sqrt(x^2 + y^2 + D^2) at every pixel (eq. 6 and the text after it)."""
    x, y = det_coords(grid)
    return D / np.sqrt(x[None, :] ** 2 + y[:, None] ** 2 + D * D)


# ------------------------------------------- O2 / O6 and their transposes
def _bin_position(grid, k):
    """Fractional s-bin index of every pixel on angle mu_k: (s_p - s_0) / ds."""
    x, y = det_coords(grid)
    mu = k * math.pi / grid.n_theta
    s_p = x[None, :] * math.cos(mu) + y[:, None] * math.sin(mu)
    return (s_p + (grid.n_s - 1) / 2.0 * grid.ds) / grid.ds


def splat_rows(img, grid):
    """sum_p img_p Lambda(t_pk - m) for all (k, m): the transpose of ``interp_rows``.

    img [nv][nu] -> [n_theta][n_s].  Each pixel deposits (1-f) on bin floor(t)
    and f on the next bin, which is exactly Lambda(t - m) for the two bins it
    touches; bins outside [0, n_s) are dropped."""
    out = np.zeros((grid.n_theta, grid.n_s))
    w = img.ravel()
    for k in range(grid.n_theta):
        t = _bin_position(grid, k).ravel()
        m0 = np.floor(t).astype(np.int64)
        f = t - m0
        for m, wt in ((m0, 1.0 - f), (m0 + 1, f)):
            ok = (m >= 0) & (m < grid.n_s)
            out[k] += np.bincount(m[ok], weights=(w * wt)[ok], minlength=grid.n_s)
    return out


def interp_rows(rows, grid):
    """sum_k sum_m rows[k][m] Lambda(t_pk - m): linear interpolation of each
    sinogram row at every pixel's s, summed over the angles.  [n_theta][n_s] -> [nv][nu]."""
    out = np.zeros((grid.nv, grid.nu))
    padded = np.zeros(grid.n_s + 2)
    for k in range(grid.n_theta):
        t = _bin_position(grid, k)
        m0 = np.floor(t).astype(np.int64)
        f = t - m0
        padded[1:-1] = rows[k]
        # index m maps to padded[m + 1]; anything outside reads a zero
        lo = np.clip(m0 + 1, 0, grid.n_s + 1)
        hi = np.clip(m0 + 2, 0, grid.n_s + 1)
        v_lo = np.where((m0 >= 0) & (m0 < grid.n_s), padded[lo], 0.0)
        v_hi = np.where((m0 + 1 >= 0) & (m0 + 1 < grid.n_s), padded[hi], 0.0)
        out += (1.0 - f) * v_lo + f * v_hi
    return out


def radon2d(img, grid):
    """A2d of one detector image as a line integral (eq. 7): (du dv/ds) splat."""
    return (grid.du * grid.dv / grid.ds) * splat_rows(img, grid)


def bp2d(rows, grid):
    """A2d^T: integral over mu in [0, pi) (eq. 8), quadrature pi/n_theta."""
    return (math.pi / grid.n_theta) * interp_rows(rows, grid)


# ------------------------------------------------ O3-O5: shift-variant filter
def d_s(a, ds):
    """Zero-padded central difference along the last axis: (a[m+1]-a[m-1]) / (2 ds)."""
    out = np.zeros_like(a)
    out[..., 1:-1] = a[..., 2:] - a[..., :-2]
    out[..., 0] = a[..., 1]
    out[..., -1] = -a[..., -2]
    return out / (2.0 * ds)


def c_geo(grid, views, v):
    """-|a'.theta| w_sino / (4 pi^2 sqrt(s^2+D^2)) folded: -|D t.n_mu + s t.l_z| / (4 pi^2 D^2).

    theta = (D n_mu + s l_z)/sqrt(s^2+D^2) is the normal of the plane through the
    source that cuts the detector in the line (s, mu) (Sec. 2.3); t = a' dlambda."""
    a, O, lx, ly, lz, D, t = view_frame(views, v)
    mu, s = radon_coords(grid)
    tn = np.cos(mu) * np.dot(t, lx) + np.sin(mu) * np.dot(t, ly)
    tz = np.dot(t, lz)
    return -np.abs(D * tn[:, None] + s[None, :] * tz) / (FOUR_PI2 * D * D)


def weight(grid, views, v, M_v, mode):
    """W = M c_geo (mode 'analytic': M is the Crofton-like factor of eq. 8/9) or
    W = M (mode 'raw': the whole redundancy weight of eq. 10 is the parameter)."""
    if mode == "raw":
        return np.asarray(M_v, np.float64)
    return np.asarray(M_v, np.float64) * c_geo(grid, views, v)


def filter_view(R_v, M_v, grid, views, v, mode="analytic"):
    """H = D( W * D R ) for one view (eqs. 7, 10, 11)."""
    Q = d_s(np.asarray(R_v, np.float64), grid.ds)
    return d_s(weight(grid, views, v, M_v, mode) * Q, grid.ds)


# ------------------------------------------------------- O7: cone-beam BP
def project_points(P, grid, views, v):
    """Fractional detector indices (i*, j*) and depth U of world points P[..., 3]."""
    a, O, lx, ly, lz, D, _ = view_frame(views, v)
    d = P - a
    U = -(d @ lz)
    i_star = (D / U) * (d @ lx) / grid.du + (grid.nu - 1) / 2.0
    j_star = (D / U) * (d @ ly) / grid.dv + (grid.nv - 1) / 2.0
    return i_star, j_star, U, D


def voxel_points(grid):
    xs = (np.arange(grid.nx) - (grid.nx - 1) / 2.0) * grid.vx + grid.ox
    ys = (np.arange(grid.ny) - (grid.ny - 1) / 2.0) * grid.vy + grid.oy
    zs = (np.arange(grid.nz) - (grid.nz - 1) / 2.0) * grid.vz + grid.oz
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def _bilinear_taps(i_star, j_star, grid):
    """The four (row, col, weight) taps of bilinear interpolation, with taps
    outside the detector given weight 0 (and a clamped, unused index)."""
    i0 = np.floor(i_star).astype(np.int64)
    j0 = np.floor(j_star).astype(np.int64)
    fi = i_star - i0
    fj = j_star - j0
    taps = []
    for dj, wj in ((0, 1.0 - fj), (1, fj)):
        for di, wi in ((0, 1.0 - fi), (1, fi)):
            ii, jj = i0 + di, j0 + dj
            ok = (ii >= 0) & (ii < grid.nu) & (jj >= 0) & (jj < grid.nv)
            taps.append((np.where(ok, jj, 0), np.where(ok, ii, 0), np.where(ok, wi * wj, 0.0)))
    return taps


def cone_bp(gF, grid, views, relu=False, points=None):
    """A3d^T with the folded weight (eq. 5, eq. 11): f(x) = sum_v (D/U)^2 bilinear(gF_v, proj_v(x)).

    gF [V][nv][nu] -> f with the shape of ``points`` (default: the voxel grid)."""
    P = voxel_points(grid) if points is None else np.asarray(points, np.float64)
    f = np.zeros(P.shape[:-1])
    for v in range(len(views)):
        i_s, j_s, U, D = project_points(P, grid, views, v)
        img = np.asarray(gF[v], np.float64)
        val = sum(w * img[jj, ii] for jj, ii, w in _bilinear_taps(i_s, j_s, grid))
        f += (D / U) ** 2 * val
    return np.maximum(f, 0.0) if relu else f


def cone_bp_literal(gF_unweighted, grid, views):
    """Paper-order variant: multiply by w_d = x^2+y^2+D^2 at pixel centres, then
    backproject with 1/|x-a|^2 (eq. 5 and eq. 11 taken literally)."""
    x, y = det_coords(grid)
    P = voxel_points(grid)
    f = np.zeros(P.shape[:-1])
    for v in range(len(views)):
        a, O, lx, ly, lz, D, _ = view_frame(views, v)
        img = np.asarray(gF_unweighted[v], np.float64) * (x[None, :] ** 2 + y[:, None] ** 2 + D * D)
        i_s, j_s, U, _ = project_points(P, grid, views, v)
        val = sum(w * img[jj, ii] for jj, ii, w in _bilinear_taps(i_s, j_s, grid))
        f += val / np.sum((P - a) ** 2, axis=-1)
    return f


# ------------------------------------------------------------- transposes
def voxel_centres(grid, idx):
    """World positions of the voxels with indices idx[n] = (iz, iy, ix), placed
    as in ``voxel_points``."""
    idx = np.asarray(idx)
    return np.stack([(idx[:, 2] - (grid.nx - 1) / 2.0) * grid.vx + grid.ox,
                     (idx[:, 1] - (grid.ny - 1) / 2.0) * grid.vy + grid.oy,
                     (idx[:, 0] - (grid.nz - 1) / 2.0) * grid.vz + grid.oz], axis=-1)


def cone_bp_adjoint(Gf, grid, views, relu_f=None, support=None):
    """Exact transpose of ``cone_bp``: every voxel spreads (D/U)^2 Gf(x) over
    its four bilinear taps.  ``relu_f`` applies the ReLU derivative mask
    [f > 0] to Gf first.

    ``support`` (optional): indices (iz, iy, ix) [n, 3] of the only voxels where
    Gf may be nonzero; Gf (and relu_f) then hold their n values, and the sum runs
    over those voxels alone (the terms of every other voxel are zero)."""
    P = voxel_points(grid) if support is None else voxel_centres(grid, support)
    G = np.asarray(Gf, np.float64)
    if relu_f is not None:
        G = G * (np.asarray(relu_f) > 0)
    out = np.zeros((len(views), grid.nv, grid.nu))
    for v in range(len(views)):
        i_s, j_s, U, D = project_points(P, grid, views, v)
        val = (D / U) ** 2 * G
        acc = np.zeros(grid.nv * grid.nu)
        for jj, ii, w in _bilinear_taps(i_s, j_s, grid):
            acc += np.bincount((jj * grid.nu + ii).ravel(), weights=(w * val).ravel(),
                               minlength=grid.nv * grid.nu)
        out[v] = acc.reshape(grid.nv, grid.nu)
    return out


def d_s_adjoint(a, ds):
    """Transpose of ``d_s``: (a[m-1] - a[m+1]) / (2 ds), zero-padded."""
    out = np.zeros_like(a)
    out[..., 1:-1] = a[..., :-2] - a[..., 2:]
    out[..., 0] = -a[..., 1]
    out[..., -1] = a[..., -2]
    return out / (2.0 * ds)


def filter_view_adjoint(GH_v, R_v, M_v, grid, views, v, mode="analytic"):
    """Transpose of H = D(W * D R) w.r.t. R and the gradient w.r.t. M.

    Returns (GM, GR): GM = (D^T GH) * (D R) * c_geo  (c_geo = 1 in 'raw' mode),
    GR = D^T( W * D^T GH )."""
    GP = d_s_adjoint(np.asarray(GH_v, np.float64), grid.ds)
    Q = d_s(np.asarray(R_v, np.float64), grid.ds)
    cg = np.ones_like(Q) if mode == "raw" else c_geo(grid, views, v)
    GM = GP * Q * cg
    GR = d_s_adjoint(weight(grid, views, v, M_v, mode) * GP, grid.ds)
    return GM, GR


def radon2d_adjoint(GR_v, grid):
    """Transpose of ``radon2d``: (du dv/ds) interp_rows."""
    return (grid.du * grid.dv / grid.ds) * interp_rows(np.asarray(GR_v, np.float64), grid)


def bp2d_adjoint(GgF_v, grid):
    """Transpose of ``bp2d``: (pi/n_theta) splat_rows."""
    return (math.pi / grid.n_theta) * splat_rows(np.asarray(GgF_v, np.float64), grid)


# -------------------------------------------------- stage-level view loops
def weight_radon(g, grid, views):
    """R_v = A2d( w_cos g_v ) for every view (eq. 7 without the derivative)."""
    return np.stack([radon2d(np.asarray(g[v], np.float64) * w_cos(grid, view_frame(views, v)[5]), grid)
                     for v in range(len(views))])


def weight_radon_adjoint(GR, grid, views):
    return np.stack([w_cos(grid, view_frame(views, v)[5]) * radon2d_adjoint(GR[v], grid)
                     for v in range(len(views))])


def filter_stack(R, M, grid, views, mode="analytic"):
    return np.stack([filter_view(R[v], M[v], grid, views, v, mode) for v in range(len(views))])


def filter_stack_adjoint(GH, R, M, grid, views, mode="analytic"):
    out = [filter_view_adjoint(GH[v], R[v], M[v], grid, views, v, mode) for v in range(len(views))]
    return np.stack([o[0] for o in out]), np.stack([o[1] for o in out])


def detector_bp(H, grid):
    return np.stack([bp2d(H[v], grid) for v in range(H.shape[0])])


def detector_bp_adjoint(GgF, grid):
    return np.stack([bp2d_adjoint(GgF[v], grid) for v in range(GgF.shape[0])])


def reconstruct(g, M, grid, views, mode="analytic", relu=False, keep=False):
    """Full eq. 12.  Returns f (and the intermediates R, H, gF when keep=True)."""
    R = weight_radon(g, grid, views)
    H = filter_stack(R, M, grid, views, mode)
    gF = detector_bp(H, grid)
    f = cone_bp(gF, grid, views, relu=relu)
    return (f, dict(R=R, H=H, gF=gF)) if keep else f


def grad_M(g, M, Gf, grid, views, mode="analytic", relu=False):
    """dL/dM given dL/df = Gf, by the chain rule through eq. 12 (f is linear in M)."""
    R = weight_radon(g, grid, views)
    f = None
    if relu:
        f = cone_bp(detector_bp(filter_stack(R, M, grid, views, mode), grid), grid, views)
    GgF = cone_bp_adjoint(Gf, grid, views, relu_f=f)
    GH = detector_bp_adjoint(GgF, grid)
    GM, _ = filter_stack_adjoint(GH, R, M, grid, views, mode)
    return GM
