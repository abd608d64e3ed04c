"""Pins of the oracle's orbit geometry, the collapsed sinogram weight c_geo and
the order of differentiation in Grangeat's function, each against something the
oracle does not compute itself.

  * eq. 9 needs, for every plane through a source point, the orbit parameters
    where the orbit crosses that plane and the orbit tangent there.  The
    crossings are checked against sign changes of the plane function on a grid
    thousands of times finer than the oracle's search, refined by bisection in
    this file; the tangent against a central difference of the orbit point and
    against the per-view tangents the view generator builds from spherical
    frames; the orbit points against the generator's source positions.  The
    weight itself is then rebuilt from those independent crossings and tangents.
  * eqs. 7 and 10 give w_sino = (s^2+D^2)/D^2 and w_red = -M |a'.theta| /
    (4 pi^2 sqrt(s^2+D^2)) for the plane through the source that cuts the
    detector in the line (s, mu) (Sec. 2.4).  The plane's normal is formed here
    from two points of that line and the source by a cross product, and the
    tangent is given large components along l_z, so the s (t.l_z) term of the
    collapsed weight is exercised.
  * eq. 6 (differentiate along u, then integrate along v) and eq. 7 (the
    discrete Radon transform first, then the s derivative) compute the same
    intermediate function; the eq. 6 side is evaluated here with the exact
    gradient of a Gaussian image and a fine quadrature along each line.
"""
import math

import numpy as np
import pytest

import synth
from oracle import crofton, pipeline as P


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


ORBITS = {
    # the benchmark workload's sinusoid (100 mm elevation amplitude, 2 periods)
    "sinusoid_c2": lambda: synth.sinusoid_orbit(24, 750.0, 1200.0, amp_mm=100.0, periods=2),
    # the paper's own sinusoid (eq. 15: 20 degrees, f = 5)
    "sinusoid_paper": lambda: synth.sinusoid_orbit(30, 750.0, 1200.0, periods=5, phi_max=math.radians(20.0)),
    "circle_arc": lambda: synth.circle_arc_orbit(10, 36, 750.0, 1200.0, 30.0),
    "circle_line": lambda: synth.circle_line_orbit(36, 11, 750.0, 1200.0, 200.0),
}


def _span(orb, seg, seam=0.0):
    """Parameter interval of a segment: one turn when closed (starting `seam`
    after the first view, so that no grid point of the dense search sits on a
    view's own parameter), else first to last view."""
    sd = orb.segs[seg]
    lo = orb.tau_of_view(seg, 0)
    if sd["closed"]:
        return lo + seam, lo + seam + 2 * math.pi
    return lo, orb.tau_of_view(seg, sd["count"] - 1)


def _dense_crossings(orb, theta, d, n=1 << 18):
    """(segment, parameter) of every sign change of a(tau).theta - d on a uniform
    grid of n intervals per segment, each refined by 100 bisection steps."""
    out = []
    for seg in range(len(orb.segs)):
        lo, hi = _span(orb, seg, seam=0.1234567)
        tau = np.linspace(lo, hi, n + 1)
        F = orb.point(seg, tau) @ theta - d
        for j in np.nonzero(np.signbit(F[:-1]) != np.signbit(F[1:]))[0]:
            a, b, fa = tau[j], tau[j + 1], F[j]
            for _ in range(100):
                mid = 0.5 * (a + b)
                fm = float(orb.point(seg, mid) @ theta - d)
                if np.signbit(fm) == np.signbit(fa):
                    a, fa = mid, fm
                else:
                    b = mid
            out.append((seg, 0.5 * (a + b)))
    return out


def _closed_turn_distance(orb, seg, t1, t2):
    d = abs(t1 - t2)
    if orb.segs[seg]["closed"]:
        d %= 2 * math.pi
        d = min(d, 2 * math.pi - d)
    return d


# ----------------------------------------------------------- orbit points
@pytest.mark.parametrize("name", list(ORBITS))
def test_orbit_points_are_the_view_sources(name):
    """The oracle's analytic orbit a(tau) at each view's parameter is the source
    position the view generator placed there (built independently, from
    spherical frames or explicit coordinates)."""
    views = ORBITS[name]()
    orb = crofton.Orbit(views)
    for v in range(len(views)):
        seg, tau = orb.locate(v)
        np.testing.assert_allclose(orb.point(seg, tau), views.src[v], rtol=0, atol=1e-9)


# -------------------------------------------------------- orbit tangents
@pytest.mark.parametrize("name", list(ORBITS))
def test_orbit_tangent_is_the_derivative_of_the_orbit_point(name):
    """a'(tau) times the per-view parameter step equals a central difference of
    a(tau) (error O(h^2) ~ 1e-10 relative) at random parameters of every segment,
    and the view generator's tangent at each view's parameter."""
    views = ORBITS[name]()
    orb = crofton.Orbit(views)
    r = np.random.Generator(np.random.PCG64(17))
    h = 1e-5
    for seg, sd in enumerate(orb.segs):
        step = {"circle": "dlam", "arc": "dphi", "line": "dz", "sinusoid": "dth"}[sd["kind"]]
        lo, hi = _span(orb, seg)
        for tau in r.uniform(lo, hi, 25):
            cd = (orb.point(seg, tau + h) - orb.point(seg, tau - h)) / (2 * h) * sd[step]
            t = orb.tangent(seg, tau)
            assert np.linalg.norm(t - cd) <= 1e-7 * np.linalg.norm(cd), (seg, tau, t, cd)
    for v in range(len(views)):
        seg, tau = orb.locate(v)
        np.testing.assert_allclose(orb.tangent(seg, tau), views.tangent[v], rtol=0,
                                   atol=1e-9 * np.linalg.norm(views.tangent[v]))


def test_orbit_taper_is_one_inside_and_ramps_to_the_floor_at_open_ends():
    """c of eq. 9: 1 on closed segments and on the middle 90 % of an open one;
    the floor at both ends; continuous and monotone on each 5 % ramp."""
    views = ORBITS["circle_arc"]()
    orb = crofton.Orbit(views)
    lo, hi = _span(orb, 0)
    u = np.linspace(0.0, 1.0, 2001)
    c = orb.taper(0, lo + u * (hi - lo))
    assert abs(c[0] - crofton.C_FLOOR) < 1e-15 and abs(c[-1] - crofton.C_FLOOR) < 1e-15
    mid = (u >= crofton.TAPER) & (u <= 1 - crofton.TAPER)
    assert np.all(c[mid] == 1.0)
    ramp = u < crofton.TAPER
    assert np.all(np.diff(c[ramp]) > 0) and np.all(np.diff(c[u > 1 - crofton.TAPER]) < 0)
    # no jump anywhere: a raised cosine's steepest step on this grid is
    # (pi/2) (1 - floor) / (0.05 * 2000) = 0.0155
    assert np.max(np.abs(np.diff(c))) < 0.016
    assert np.all(orb.taper(1, np.linspace(0, 2 * math.pi, 50)) == 1.0)


# ------------------------------------------------------------ crossings
@pytest.mark.parametrize("name", list(ORBITS))
def test_plane_orbit_crossings_match_dense_sign_changes(name):
    """Every crossing of a plane with the orbit (eq. 9's sum runs over them):
    random planes, and planes through random orbit points (the planes eq. 9
    evaluates), against sign changes on a grid of 2^18 intervals per segment."""
    views = ORBITS[name]()
    orb = crofton.Orbit(views)
    r = np.random.Generator(np.random.PCG64(23))
    for trial in range(24):
        th = r.normal(size=3)
        th /= np.linalg.norm(th)
        if trial % 2:
            d = float(r.uniform(-500.0, 500.0))
        else:
            seg = int(r.integers(len(orb.segs)))
            lo, hi = _span(orb, seg)
            d = float(orb.point(seg, r.uniform(lo + 0.01 * (hi - lo), hi - 0.01 * (hi - lo))) @ th)
        got = orb.intersections(th, d)
        ref = _dense_crossings(orb, th, d)
        assert len(got) == len(ref), (trial, got, ref)
        for seg, tau in ref:
            dist = min((_closed_turn_distance(orb, seg, tau, t2) for s2, t2 in got if s2 == seg), default=9.0)
            assert dist < 1e-9, (trial, seg, tau, got)


def _M_from_dense_crossings(orb, views, grid, v, bins):
    """Eq. 9 rebuilt from the dense crossings and a central-difference tangent."""
    seg_v, tau_v = orb.locate(v)
    a, O, lx, ly, lz, D, _ = P.view_frame(views, v)
    mu, s = P.radon_coords(grid)
    step = {"circle": "dlam", "arc": "dphi", "line": "dz", "sinusoid": "dth"}
    h = 1e-6

    def tangent(seg, tau):
        sd = orb.segs[seg]
        return (orb.point(seg, tau + h) - orb.point(seg, tau - h)) / (2 * h) * sd[step[sd["kind"]]]

    out = []
    for k, m in bins:
        n = math.cos(mu[k]) * lx + math.sin(mu[k]) * ly
        th = (D * n + s[m] * lz) / math.hypot(s[m], D)
        hits = _dense_crossings(orb, th, float(a @ th), n=1 << 16)
        # the plane holds a(tau_v) by construction; at the end of an open segment
        # the grid starts on that root, where no sign change is seen
        if not any(sg == seg_v and _closed_turn_distance(orb, sg, t, tau_v) < 1e-9 for sg, t in hits):
            hits.append((seg_v, tau_v))
        w = [abs(float(tangent(sg, t) @ th)) ** 2 * float(orb.taper(sg, t)) for sg, t in hits]
        num = abs(float(tangent(seg_v, tau_v) @ th)) ** 2 * float(orb.taper(seg_v, tau_v))
        out.append(num / sum(w))
    return np.array(out)


@pytest.mark.parametrize("name", ["sinusoid_c2", "sinusoid_paper", "circle_arc"])
def test_crofton_weight_from_independent_crossings_and_tangents(name):
    """M of eq. 9 on Radon-grid planes of several views equals the same ratio
    formed from the dense crossings and central-difference tangents above (a
    missed or spurious crossing, or a wrong tangent component, changes M)."""
    views = ORBITS[name]()
    orb = crofton.Orbit(views)
    grid = synth.Grid(nu=40, nv=40, du=4.0, dv=4.0, n_theta=12, n_s=57, ds=4.0,
                      nx=1, ny=1, nz=1, vx=1, vy=1, vz=1)
    r = np.random.Generator(np.random.PCG64(29))
    for v in (0, len(views) // 3, len(views) - 2):
        bins = [(int(r.integers(grid.n_theta)), int(r.integers(grid.n_s))) for _ in range(6)]
        cg = P.c_geo(grid, views, v)
        bins = [b for b in bins if abs(cg[b]) > 1e-6 * np.abs(cg).max()]   # skip planes tangent to the orbit
        got = crofton.M_view(views, grid, v, bins=bins)
        ref = _M_from_dense_crossings(orb, views, grid, v, bins)
        np.testing.assert_allclose(got, ref, rtol=1e-7, atol=1e-12)


# ---------------------------------------------------------- c_geo (eq. 10)
def test_collapsed_sinogram_weight_from_the_plane_through_the_detector_line():
    """c_geo = w_sino w_red / M with theta the unit normal of the plane through the
    source and the detector line (s, mu), formed by a cross product, for
    tangents with large components along l_z (|t.l_z| up to |t.l_x|)."""
    grid = synth.Grid(nu=30, nv=24, du=1.3, dv=1.1, n_theta=10, n_s=41, ds=1.3,
                      nx=1, ny=1, nz=1, vx=1, vy=1, vz=1)
    views = synth.random_nn_orbit(6, 750.0, 1200.0, seed=4)
    r = np.random.Generator(np.random.PCG64(31))
    for v in range(len(views)):
        lz = np.cross(views.ex[v], views.ey[v])
        t = r.normal(0, 8, 3)
        views.tangent[v] = t - (t @ lz) * lz + r.choice([-1.0, 1.0]) * r.uniform(4, 10) * lz
    mu, s = P.radon_coords(grid)
    for v in range(len(views)):
        a = views.src[v]
        O = views.det_center[v]
        lx, ly = views.ex[v], views.ey[v]
        lz = np.cross(lx, ly)
        D = float(np.dot(a - O, lz))
        t = views.tangent[v]
        assert abs(t @ lz) > 0.05 * np.linalg.norm(t)
        c = P.c_geo(grid, views, v)
        for k in range(grid.n_theta):
            n = math.cos(mu[k]) * lx + math.sin(mu[k]) * ly
            n_perp = -math.sin(mu[k]) * lx + math.cos(mu[k]) * ly
            for m in range(grid.n_s):
                p1 = O + s[m] * n              # foot of the perpendicular from the detector centre
                p2 = p1 + 7.0 * n_perp         # a second point of the same detector line
                th = np.cross(p1 - a, p2 - a)
                th /= np.linalg.norm(th)
                w_sino = (s[m] ** 2 + D * D) / (D * D)
                w_red = -abs(float(t @ th)) / (4 * math.pi ** 2 * math.sqrt(s[m] ** 2 + D * D))
                # the cross product of 1200 mm vectors rounds at ~1e-13 of |t| / (4 pi^2 D)
                assert abs(c[k, m] - w_sino * w_red) <= 1e-10 * np.abs(c).max(), (v, k, m)


# --------------------------------------------------- eq. 6 against eq. 7
def test_grangeat_function_integrate_then_differentiate_equals_eq6():
    """S(s, mu) = w_sino d/ds A2d(w_cos g) (eq. 7) against
    S = w_sino int dv d/du (D g / sqrt(u^2+v^2+D^2)) at u = s (eq. 6), for a Gaussian
    g whose gradient is known in closed form.  D is short (30 pixels) and the
    blob sits 15 pixels off centre, so w_cos changes the result by 17 % (leaving
    it out fails the bound); the remaining 0.8 % is the central difference's
    O(ds^2) error.  The pixel-driven Radon transform ripples at mu = 45 and 135
    degrees (see the Radon pin), where only a loose bound applies."""
    N = 112
    grid = synth.Grid(nu=N, nv=N, du=1.0, dv=1.0, n_theta=36, n_s=synth.radon_bins(N, N), ds=1.0,
                      nx=1, ny=1, nz=1, vx=1, vy=1, vz=1)
    D = 30.0
    x0, y0, sig = 12.0, -9.0, 8.0
    x, y = P.det_coords(grid)
    img = np.exp(-((x[None, :] - x0) ** 2 + (y[:, None] - y0) ** 2) / (2 * sig * sig))
    mu, s = P.radon_coords(grid)
    w_sino = (s ** 2 + D * D) / (D * D)
    S7 = w_sino[None, :] * P.d_s(P.radon2d(img * P.w_cos(grid, D), grid), grid.ds)

    v = np.linspace(-N, N, 20001)               # the blob is below 1e-6 at the detector's edges
    S6 = np.zeros_like(S7)
    for k, m_ in enumerate(mu):
        c, sn = math.cos(m_), math.sin(m_)
        X = s[:, None] * c - v[None, :] * sn
        Y = s[:, None] * sn + v[None, :] * c
        gg = np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2 * sig * sig))
        rho = np.sqrt(X * X + Y * Y + D * D)
        gx, gy = -(X - x0) / sig ** 2 * gg, -(Y - y0) / sig ** 2 * gg
        hx = D * gx / rho - D * gg * X / rho ** 3
        hy = D * gy / rho - D * gg * Y / rho ** 3
        S6[k] = w_sino * np.trapezoid(hx * c + hy * sn, v, axis=1)   # d/du at fixed v, then int dv
    diag = np.minimum(np.abs(np.degrees(mu) - 45), np.abs(np.degrees(mu) - 135)) < 3
    assert rel(S7[~diag], S6[~diag]) < 1.2e-2
    assert rel(S7[diag], S6[diag]) < 0.5
