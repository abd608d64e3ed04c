"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test ties one oracle function to something other than its own formula:
closed-form transforms, exact special cases, adjoint identities, the FDK
equivalence on a circle, exact reconstruction of a uniform ball where the
orbit satisfies Tuy's condition, Crofton partitions of unity, Siddon chord
lengths, and finite differences.  A plausible slip (dropped term, wrong sign or
index, transposed operand, wrong scale) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from synth.phantom import (ball, gaussian_blobs, project_ellipsoids, project_gaussian_blobs,
                           voxelize, voxelize_gaussian_blobs)
from oracle import crofton, fdk, pipeline as P, siddon

HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def small_grid(nu=20, nv=17, n_theta=13, n_s=None, nx=9, ny=8, nz=7, du=1.0, dv=1.0, ds=None, vox=1.5):
    return synth.Grid(nu=nu, nv=nv, du=du, dv=dv, n_theta=n_theta,
                      n_s=n_s or synth.radon_bins(nu, nv), ds=ds or du,
                      nx=nx, ny=ny, nz=nz, vx=vox, vy=vox * 0.9, vz=vox * 1.1, ox=0.3, oy=-0.2, oz=0.1)


# --------------------------------------------------------------- 2D Radon
def test_radon_of_offset_gaussian_matches_closed_form():
    """A2d of exp(-|p-p0|^2/(2 sig^2)) is sig sqrt(2 pi) exp(-(s - p0.n_mu)^2/(2 sig^2)).
    An offset centre makes a sign slip in sin(mu) or an x/y swap visible.

    The pixel-driven splat has a moire ripple near mu = 45 and 135 degrees (pixel
    centres project at spacing ds/sqrt(2) there), so the tight bound is taken on
    the other angles and the diagonal ones only get a loose bound; the integral
    over s is checked exactly at every angle."""
    g = synth.Grid(nu=64, nv=64, du=1.0, dv=1.0, n_theta=36, n_s=91, ds=1.0,
                   nx=1, ny=1, nz=1, vx=1, vy=1, vz=1)
    x, y = P.det_coords(g)
    x0, y0, sig = 3.0, -5.0, 6.0
    img = np.exp(-((x[None, :] - x0) ** 2 + (y[:, None] - y0) ** 2) / (2 * sig * sig))
    R = P.radon2d(img, g)
    mu, s = P.radon_coords(g)
    s0 = x0 * np.cos(mu) + y0 * np.sin(mu)
    ref = sig * math.sqrt(2 * math.pi) * np.exp(-(s[None, :] - s0[:, None]) ** 2 / (2 * sig * sig))
    diag = np.minimum(np.abs(np.degrees(mu) - 45), np.abs(np.degrees(mu) - 135)) < 10
    assert rel(R[~diag], ref[~diag]) < 4e-3
    assert rel(R[diag], ref[diag]) < 0.1
    # mass: int R ds = int int g dx dy at every angle, exactly
    np.testing.assert_allclose(R.sum(axis=1) * g.ds, img.sum() * g.du * g.dv, rtol=1e-12)


def test_radon_axis_aligned_angles_are_exact_column_and_row_sums():
    """At mu = 0 (and pi/2) every pixel centre lands on a bin centre when the grids
    are aligned, so the line integral is exactly dv x column sum (du x row sum)."""
    g = synth.Grid(nu=15, nv=13, du=1.0, dv=1.0, n_theta=4, n_s=21, ds=1.0,
                   nx=1, ny=1, nz=1, vx=1, vy=1, vz=1)
    img = synth.rand_array((13, 15), seed=3).astype(np.float64)
    R = P.radon2d(img, g)
    off_u = (g.n_s - 1) // 2 - (g.nu - 1) // 2
    off_v = (g.n_s - 1) // 2 - (g.nv - 1) // 2
    col = g.dv * img.sum(axis=0)
    row = g.du * img.sum(axis=1)
    np.testing.assert_allclose(R[0, off_u:off_u + g.nu], col, rtol=0, atol=1e-13)
    np.testing.assert_allclose(R[2, off_v:off_v + g.nv], row, rtol=0, atol=1e-13)
    assert abs(R[0].sum() - col.sum()) < 1e-12


def test_detector_bp_of_constant_rows_is_pi_times_constant():
    """int_0^pi c dmu = pi c at every pixel (all pixel s values lie inside the s grid)."""
    g = small_grid()
    rows = np.full((g.n_theta, g.n_s), 2.5)
    np.testing.assert_allclose(P.bp2d(rows, g), math.pi * 2.5, rtol=1e-14)


def test_central_difference_exact_on_quadratics_and_antisymmetric():
    ds = 0.7
    s = np.arange(11) * ds
    q = 1.3 - 0.4 * s + 0.25 * s * s
    d = P.d_s(q, ds)
    np.testing.assert_allclose(d[1:-1], (-0.4 + 0.5 * s)[1:-1], rtol=0, atol=1e-13)
    n = 9
    Dm = np.stack([P.d_s(e, ds) for e in np.eye(n)], axis=1)
    Dt = np.stack([P.d_s_adjoint(e, ds) for e in np.eye(n)], axis=1)
    np.testing.assert_allclose(Dt, Dm.T, atol=1e-15)
    np.testing.assert_allclose(Dm.T, -Dm, atol=1e-15)


# ----------------------------------------------------- weights / geometry
def test_circle_redundancy_weight_matches_eq14_closed_form():
    """On a circle t = R dlam l_x and t.l_z = 0, so w_red w_sino = -M R |cos mu| dlam / (4 pi^2 D):
    eq. 14's |a'.theta| with the R*D factor that a(lambda) = R(cos, sin, 0) gives
    (the printed D^2 would equal it only for R = D)."""
    g = small_grid(n_theta=24)
    V = 12
    views = synth.circle_orbit(V, 750.0, 1200.0)
    mu, _ = P.radon_coords(g)
    for v in (0, 5):
        c = P.c_geo(g, views, v)
        ref = -750.0 * (2 * math.pi / V) * np.abs(np.cos(mu)) / (4 * math.pi ** 2 * 1200.0)
        np.testing.assert_allclose(c, np.broadcast_to(ref[:, None], c.shape), rtol=1e-12, atol=1e-18)


def test_projection_of_points_on_pixel_rays_and_wd_identity():
    """A point at depth U on the ray through pixel (i, j) projects back to (i, j), and
    w_d(P)/|x-a|^2 equals the folded D^2/U^2 weight there (eq. 5 with eq. 11)."""
    g = small_grid()
    views = synth.sinusoid_orbit(8, 750.0, 1200.0)
    rng = np.random.Generator(np.random.PCG64(5))
    x, y = P.det_coords(g)
    for v in range(3):
        a, O, lx, ly, lz, D, _ = P.view_frame(views, v)
        i, j = rng.integers(0, g.nu, 20), rng.integers(0, g.nv, 20)
        Pd = O + x[i, None] * lx + y[j, None] * ly
        U = rng.uniform(600, 900, 20)
        X = a + (U / D)[:, None] * (Pd - a)
        i_s, j_s, U2, D2 = P.project_points(X, g, views, v)
        np.testing.assert_allclose(i_s, i, atol=1e-9)
        np.testing.assert_allclose(j_s, j, atol=1e-9)
        np.testing.assert_allclose(U2, U, rtol=1e-12)
        wd = x[i] ** 2 + y[j] ** 2 + D * D
        np.testing.assert_allclose(wd / np.sum((X - a) ** 2, axis=1), D * D / U ** 2, rtol=1e-12)


def test_folded_and_literal_detector_weight_agree_to_discretisation_level():
    g = small_grid(nu=48, nv=40, nx=10, ny=10, nz=10, vox=1.0)
    views = synth.circle_orbit(6, 750.0, 1200.0)
    x, y = P.det_coords(g)
    gF = np.stack([np.exp(-(x[None, :] - 2) ** 2 / 60 - (y[:, None] + 1) ** 2 / 80)] * len(views))
    a = P.cone_bp(gF, g, views)
    b = P.cone_bp_literal(gF, g, views)
    assert rel(a, b) < 1e-3


# ----------------------------------------------------- adjoint identities
@pytest.mark.parametrize("pair", ["radon", "bp2d", "filter_R", "filter_M", "filter_M_raw", "cone",
                                  "weight_radon"])
def test_adjoint_identity(pair):
    g = small_grid()
    views = synth.sinusoid_orbit(5, 750.0, 1200.0)
    # give one view a tangent with a component along l_z so the s*t.l_z term is exercised
    views.tangent[2] += 3.0 * np.cross(views.ex[2], views.ey[2])
    r = np.random.Generator(np.random.PCG64(11))
    V, K, S = len(views), g.n_theta, g.n_s
    if pair == "radon":
        x, y = r.normal(size=(g.nv, g.nu)), r.normal(size=(K, S))
        lhs, rhs = np.vdot(P.radon2d(x, g), y), np.vdot(x, P.radon2d_adjoint(y, g))
    elif pair == "bp2d":
        x, y = r.normal(size=(K, S)), r.normal(size=(g.nv, g.nu))
        lhs, rhs = np.vdot(P.bp2d(x, g), y), np.vdot(x, P.bp2d_adjoint(y, g))
    elif pair.startswith("filter"):
        mode = "raw" if pair.endswith("raw") else "analytic"
        Rv, Mv, GH = r.normal(size=(K, S)), r.normal(size=(K, S)), r.normal(size=(K, S))
        GM, GR = P.filter_view_adjoint(GH, Rv, Mv, g, views, 2, mode)
        if pair == "filter_R":
            lhs, rhs = np.vdot(P.filter_view(Rv, Mv, g, views, 2, mode), GH), np.vdot(Rv, GR)
        else:
            lhs, rhs = np.vdot(P.filter_view(Rv, Mv, g, views, 2, mode), GH), np.vdot(Mv, GM)
    elif pair == "cone":
        x, y = r.normal(size=(V, g.nv, g.nu)), r.normal(size=(g.nz, g.ny, g.nx))
        lhs, rhs = np.vdot(P.cone_bp(x, g, views), y), np.vdot(x, P.cone_bp_adjoint(y, g, views))
    else:
        x, y = r.normal(size=(V, g.nv, g.nu)), r.normal(size=(V, K, S))
        lhs, rhs = np.vdot(P.weight_radon(x, g, views), y), np.vdot(x, P.weight_radon_adjoint(y, g, views))
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), 1e-300) + 1e-12


# --------------------------------------------------- whole-chain exactness
def test_circle_with_half_weight_reduces_to_fdk():
    """For a circle with M = 1/2 the chain A2d^T W D^2 A2d equals (R dlam/2D) times a
    ramp filter along u, i.e. Feldkamp's formula.  Compared with the independent
    textbook FDK and with the voxelised smooth phantom; a wrong R/D factor, a
    lost 2 or pi, or a sign flip moves the scale far outside these bounds."""
    g = synth.Grid(nu=64, nv=64, du=1.0, dv=1.0, n_theta=90, n_s=91, ds=1.0,
                   nx=20, ny=20, nz=20, vx=1.0, vy=1.0, vz=1.0)
    views = synth.circle_orbit(72, 750.0, 1200.0)
    bl = gaussian_blobs(3, 20, seed=7, sigma_range=(2.5, 3.5))
    gp = project_gaussian_blobs(bl, g, views)
    M = np.full((len(views), g.n_theta, g.n_s), 0.5)
    f_dc = P.reconstruct(gp, M, g, views)
    f_fdk = fdk.fdk_circle(gp, g, views)
    gt = voxelize_gaussian_blobs(bl, g)
    assert rel(f_dc, f_fdk) < 0.06
    assert rel(f_fdk, gt) < 0.02
    scale = float((f_dc * gt).sum() / (gt * gt).sum())
    assert 0.96 < scale < 1.01


def _ball_points(zc, zs, half=2.5):
    xs = np.linspace(-half, half, 6)
    X, Y = np.meshgrid(xs, xs)
    return np.stack([np.stack([X, Y, np.full_like(X, z)], -1) for z in zs])


def test_uniform_ball_midplane_exact_on_circle():
    """Every plane through a mid-plane point meets the circle twice, so with M = 1/2
    the mid-plane of a uniform ball is reconstructed exactly up to discretisation."""
    g = synth.Grid(nu=64, nv=64, du=1.0, dv=1.0, n_theta=120, n_s=91, ds=1.0,
                   nx=1, ny=1, nz=1, vx=1, vy=1, vz=1)
    views = synth.circle_orbit(90, 750.0, 1200.0)
    gp = project_ellipsoids(ball([0, 0, 0], 6.0), g, views).numpy()
    M = np.full((len(views), g.n_theta, g.n_s), 0.5)
    gF = P.detector_bp(P.filter_stack(P.weight_radon(gp, g, views), M, g, views), g)
    f = P.cone_bp(gF, g, views, points=_ball_points(0.0, [0.0]))
    assert abs(f.mean() - 1.0) < 0.01 and f.std() < 0.01


def test_uniform_ball_off_midplane_exact_on_circle_plus_line_with_crofton_weight():
    """Circle + line satisfies Tuy's condition for the ball; with the eq. 9 weight
    the reconstruction is exact everywhere, while the circle alone is not."""
    N = 112
    g = synth.Grid(nu=N, nv=N, du=1.2, dv=1.2, n_theta=120, n_s=synth.radon_bins(N, N), ds=1.2,
                   nx=1, ny=1, nz=1, vx=1, vy=1, vz=1)
    zc = 9.0
    pts = _ball_points(zc, [zc - 3, zc, zc + 3])
    b = ball([0, 0, zc], 6.0)
    means = {}
    for kind in ("circle", "circle_line"):
        views = (synth.circle_orbit(90, 100.0, 200.0) if kind == "circle"
                 else synth.circle_line_orbit(90, 41, 100.0, 200.0, half_len=32.0))
        gp = project_ellipsoids(b, g, views).numpy()
        M = np.stack([crofton.M_view_closed_form(views, g, v) for v in range(len(views))])
        gF = P.detector_bp(P.filter_stack(P.weight_radon(gp, g, views), M, g, views), g)
        f = P.cone_bp(gF, g, views, points=pts)
        means[kind] = f.reshape(3, -1).mean(axis=1)
    assert np.all(np.abs(means["circle_line"] - 1.0) < 3e-3), means
    assert abs(means["circle"][2] - 1.0) > 3 * abs(means["circle_line"][2] - 1.0), means


# ------------------------------------------------------ Crofton weight (eq. 9)
def test_crofton_weight_is_one_half_on_a_circle():
    g = small_grid(n_theta=16)
    views = synth.circle_orbit(36, 750.0, 1200.0)
    M = crofton.M_view_closed_form(views, g, 4)
    cg = P.c_geo(g, views, 4)
    generic = crofton.M_view(views, g, 4, bins=[(1, 3), (7, 10), (12, 0)])
    np.testing.assert_allclose(M[np.abs(cg) > 1e-9], 0.5, rtol=1e-12)
    np.testing.assert_allclose(generic, 0.5, rtol=1e-12)


@pytest.mark.parametrize("orbit", ["sinusoid", "circle_arc", "circle_line"])
def test_crofton_partition_of_unity(orbit):
    """Summing eq. 9 over all intersections of one plane with the orbit gives 1."""
    if orbit == "sinusoid":
        views = synth.sinusoid_orbit(24, 750.0, 1200.0, amp_mm=100.0, periods=2)
    elif orbit == "circle_arc":
        views = synth.circle_arc_orbit(10, 36, 750.0, 1200.0, 30.0)
    else:
        views = synth.circle_line_orbit(36, 11, 750.0, 1200.0, 200.0)
    orb = crofton.Orbit(views)
    r = np.random.Generator(np.random.PCG64(21))
    checked = 0
    for _ in range(12):
        v = int(r.integers(len(views)))
        seg, tau = orb.locate(v)
        th = r.normal(size=3)
        th /= np.linalg.norm(th)
        d = float(orb.point(seg, tau) @ th)
        hits = orb.intersections(th, d)
        assert any(abs(s_ - seg) == 0 and abs(t_ - tau) < 1e-9 for s_, t_ in hits) or \
            any(np.linalg.norm(orb.point(s_, t_) - orb.point(seg, tau)) < 1e-6 for s_, t_ in hits)
        tot = sum(crofton.M_point(orb, s_, t_, th) for s_, t_ in hits)
        assert abs(tot - 1.0) < 1e-10
        checked += 1
    assert checked == 12


def test_crofton_open_circle_counts_only_covered_parameters():
    """Eq. 9 sums over source positions of the orbit: on a half circle a plane
    whose second crossing of the full circle lies on the missing half meets the
    orbit once, so the weight of the view it passes through is 1."""
    views = synth.circle_orbit(64, 750.0, 1200.0, start=0.0, span=math.pi)
    orb = crofton.Orbit(views)
    assert not orb.segs[0]["closed"]
    seg, tau = orb.locate(32)                       # lambda = pi / 2, mid-segment (taper 1)
    th = np.array([1.0, 0.05, 0.0]) / math.hypot(1.0, 0.05)
    d = float(orb.point(seg, tau) @ th)
    hits = orb.intersections(th, d)
    assert len(hits) == 1                           # the full circle's other crossing is at -84.3 deg
    assert crofton.M_point(orb, seg, tau, th) == 1.0
    # with the normal turned so both crossings lie on the half circle, they share the weight
    th2 = np.array([0.6, 0.8, 0.0])
    hits2 = orb.intersections(th2, float(orb.point(seg, tau) @ th2))
    assert len(hits2) == 2
    assert abs(sum(crofton.M_point(orb, s_, t_, th2) for s_, t_ in hits2) - 1.0) < 1e-12
    # every plane through the first or the last source point crosses the orbit
    # there, and the weights of its crossings sum to 1
    views = synth.circle_orbit(40, 750.0, 1200.0, start=0.3, span=math.pi)
    orb = crofton.Orbit(views)
    r = np.random.Generator(np.random.PCG64(9))
    for v in (0, 39):
        seg, tau = orb.locate(v)
        for _ in range(200):
            th = r.normal(size=3)
            th /= np.linalg.norm(th)
            hits = orb.intersections(th, float(orb.point(seg, tau) @ th))
            assert any(abs(t_ - tau) < 1e-9 for _, t_ in hits)
            assert abs(sum(crofton.M_point(orb, s_, t_, th) for s_, t_ in hits) - 1.0) < 1e-10
    # the vectorised closed form agrees with the per-bin search on this orbit,
    # wherever the filter uses the weight (on planes tangent to the orbit at every
    # crossing eq. 9 is 0/0, the 1/n fallback depends on rounding, and c_geo = 0)
    g = small_grid(n_theta=12)
    bins = [(k, m) for k in range(0, 12, 3) for m in range(0, g.n_s, 4)]
    for v in (0, 3, 20, 39):
        Mc = crofton.M_view_closed_form(views, g, v)
        Mg = crofton.M_view(views, g, v, bins=bins)
        cg = P.c_geo(g, views, v)
        used = np.array([abs(cg[k, m]) > 1e-9 * np.abs(cg).max() for k, m in bins])
        assert used.sum() >= 0.7 * len(bins)       # one angle row of the grid is tangent
        np.testing.assert_allclose(np.array([Mc[k, m] for k, m in bins])[used], Mg[used], rtol=1e-10, atol=1e-12)


def test_crofton_intersection_count_matches_brute_force_polyline():
    views = synth.circle_line_orbit(36, 11, 750.0, 1200.0, 200.0)
    orb = crofton.Orbit(views)
    r = np.random.Generator(np.random.PCG64(8))
    for _ in range(20):
        th = r.normal(size=3)
        th /= np.linalg.norm(th)
        d = float(r.uniform(-300, 300))
        n_closed = len(orb.intersections(th, d))
        n_brute = 0
        for seg, sd in enumerate(orb.segs):
            lo = orb.tau_of_view(seg, 0)
            hi = lo + 2 * math.pi if sd["kind"] == "circle" else orb.tau_of_view(seg, sd["count"] - 1)
            tau = np.linspace(lo, hi, 200001)
            F = orb.point(seg, tau) @ th - d
            n_brute += int(np.sum(np.sign(F[:-1]) != np.sign(F[1:])))
        assert n_closed == n_brute


# ----------------------------------------------------------------- Siddon
def test_siddon_chord_through_uniform_box_and_single_voxel():
    g = synth.Grid(nu=1, nv=1, du=1, dv=1, n_theta=1, n_s=1, ds=1, nx=7, ny=5, nz=6,
                   vx=1.0, vy=1.5, vz=0.8, ox=0.2, oy=-0.3, oz=0.1)
    ones = np.ones((g.nz, g.ny, g.nx))
    r = np.random.Generator(np.random.PCG64(2))
    lo = np.array([-3.5 + 0.2, -3.75 - 0.3, -2.4 + 0.1])
    hi = np.array([3.5 + 0.2, 3.75 - 0.3, 2.4 + 0.1])
    for _ in range(25):
        p0 = r.uniform(-20, 20, 3)
        p1 = r.uniform(-20, 20, 3)
        d = p1 - p0
        with np.errstate(divide="ignore"):
            t1, t2 = (lo - p0) / d, (hi - p0) / d
        tin = max(0.0, np.max(np.minimum(t1, t2)))
        tout = min(1.0, np.min(np.maximum(t1, t2)))
        ref = max(0.0, tout - tin) * np.linalg.norm(d)
        assert abs(siddon.project_rays(ones, g, p0, p1)[0] - ref) < 1e-10
    one = np.zeros((g.nz, g.ny, g.nx))
    one[2, 3, 4] = 1.0
    c = np.array([(4 - 3) * 1.0 + 0.2, (3 - 2) * 1.5 - 0.3, (2 - 2.5) * 0.8 + 0.1])
    assert abs(siddon.project_rays(one, g, c - [0, 0, 30], c + [0, 0, 30])[0] - 0.8) < 1e-12


def test_siddon_of_voxelised_ball_is_close_to_analytic_chords():
    g = synth.Grid(nu=24, nv=24, du=1.6, dv=1.6, n_theta=1, n_s=1, ds=1,
                   nx=40, ny=40, nz=40, vx=0.5, vy=0.5, vz=0.5)
    views = synth.circle_orbit(3, 750.0, 1200.0)
    b = ball([1.0, -0.5, 0.5], 7.0)
    vol = voxelize(b, g)
    s = siddon.project(vol, g, views)
    a = project_ellipsoids(b, g, views).numpy()
    core = a > 0.5 * a.max()          # rays well inside the ball; edge rays see the voxel staircase
    assert rel(s[core], a[core]) < 0.03
    assert abs(s.max() - a.max()) < 0.02 * a.max()


# --------------------------------------------------------------- gradients
def test_gradient_matches_finite_differences():
    """f is linear in M and the loss is quadratic, so a central difference along a
    one-view direction equals <dL/dM, delta> up to rounding."""
    g = small_grid(nu=18, nv=14, n_theta=10, nx=7, ny=6, nz=6)
    views = synth.circle_arc_orbit(3, 5, 750.0, 1200.0, 30.0)
    r = np.random.Generator(np.random.PCG64(4))
    gp = r.uniform(0, 1, (len(views), g.nv, g.nu))
    M = r.uniform(0.2, 0.8, (len(views), g.n_theta, g.n_s))
    target = r.normal(size=(g.nz, g.ny, g.nx)) * 1e-4
    loss = lambda MM: 0.5 * np.sum((P.reconstruct(gp, MM, g, views) - target) ** 2)
    Gf = P.reconstruct(gp, M, g, views) - target
    GM = P.grad_M(gp, M, Gf, g, views)
    delta = np.zeros_like(M)
    delta[3] = r.normal(size=M.shape[1:])
    h = 1e-3
    fd = (loss(M + h * delta) - loss(M - h * delta)) / (2 * h)
    assert abs(fd - np.vdot(GM, delta)) <= 1e-8 * abs(fd)


# ------------------------------------------------------ paper's geometry
def test_paper_geometry_fixture_and_radon_bin_rule():
    with open(os.path.join(HERE, "golden", "paper_geometry.json")) as fh:
        gold = json.load(fh)
    det = gold["table2_parallel_beam"]
    assert synth.radon_bins(det["detector_u"], det["detector_v"]) == det["radon_bins"]
    for cfg, n in (("C1", 91), ("C2", 725), ("C5", 1381)):
        d = synth.CONFIGS[cfg]["det"]
        assert synth.radon_bins(d, d) == n


@pytest.mark.parametrize("orbit", ["circle", "sinusoid", "circle_arc", "circle_line"])
def test_orbit_frames(orbit):
    if orbit == "circle":
        views = synth.circle_orbit(40, 750.0, 1200.0)
    elif orbit == "sinusoid":
        views = synth.sinusoid_orbit(400, 750.0, 1200.0)
    elif orbit == "circle_arc":
        views = synth.circle_arc_orbit(100, 360, 750.0, 1200.0)
    else:
        views = synth.circle_line_orbit(40, 9, 750.0, 1200.0, 30.0)
    lz = np.cross(views.ex, views.ey)
    np.testing.assert_allclose(np.einsum("ij,ij->i", views.ex, views.ey), 0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(lz, axis=1), 1, atol=1e-12)
    D = np.einsum("ij,ij->i", views.src - views.det_center, lz)
    np.testing.assert_allclose(D, 1200.0, rtol=1e-12)
    np.testing.assert_allclose(views.src - views.det_center, D[:, None] * lz, atol=1e-9)
    if orbit in ("circle", "sinusoid"):     # closed: tangent ~ central difference of positions
        cd = 0.5 * (np.roll(views.src, -1, 0) - np.roll(views.src, 1, 0))
        assert rel(cd, views.tangent) < 1e-2   # central difference is off by ~dlam^2/6


def test_cone_adjoint_restricted_to_a_support_is_the_dense_sum():
    """The support form of the cone transpose (used where the full volume is too
    large for the oracle) sums the same terms as the dense form of a volume that
    is zero off the support, with the ReLU mask applied to the same values."""
    g, views = synth.config_geometry("C1", n_views=5)
    r = np.random.Generator(np.random.PCG64(1))
    idx = np.unique(np.stack([r.integers(0, n, 300) for n in (g.nz, g.ny, g.nx)], 1), axis=0)
    vals, fr = r.normal(size=len(idx)), r.normal(size=len(idx))
    Gf, F = np.zeros((g.nz, g.ny, g.nx)), np.zeros((g.nz, g.ny, g.nx))
    Gf[idx[:, 0], idx[:, 1], idx[:, 2]] = vals
    F[idx[:, 0], idx[:, 1], idx[:, 2]] = fr
    dense = P.cone_bp_adjoint(Gf, g, views, relu_f=F)
    np.testing.assert_allclose(P.cone_bp_adjoint(vals, g, views, relu_f=fr, support=idx), dense,
                               rtol=1e-13, atol=1e-13 * np.abs(dense).max())
