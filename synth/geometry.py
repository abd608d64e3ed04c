"""Scan geometry: sampling grids and source orbits with their detector frames.

Conventions (shared vocabulary, not method code):
  * world frame in mm, isocentre at the origin;
  * detector frame per view (paper, Fig. 1): origin O at the detector centre,
    unit vectors l_x, l_y in the detector plane and l_z = l_x x l_y pointing
    towards the source; the source sits on the detector normal through O at
    distance D (the source-detector distance);
  * l_x is the horizontal direction of source motion, l_y = l_z x l_x;
  * the orbit tangent is stored already multiplied by the view spacing,
    t = a'(lambda) * dlambda  (mm), so a sum over views needs no further
    quadrature weight.

Orbits follow the paper's experiments: circle (Sec. 4.1), sinusoid (eq. 15,
Sec. 4.2), circle plus arc (Sec. 4.3), random nearest-neighbour (Sec. 4.4), and
a circle plus line orbit used for exactness checks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np


@dataclass
class Grid:
    """Sampling of detector, Radon plane and volume (all lengths in mm)."""
    nu: int
    nv: int
    du: float
    dv: float
    n_theta: int
    n_s: int
    ds: float
    nx: int
    ny: int
    nz: int
    vx: float
    vy: float
    vz: float
    ox: float = 0.0
    oy: float = 0.0
    oz: float = 0.0

    def as_dict(self):
        return asdict(self)

    @property
    def nvox(self):
        return self.nx * self.ny * self.nz


def radon_bins(nu: int, nv: int) -> int:
    """Number of s bins that covers the detector diagonal at spacing du.

    Reproduces the paper's 785 bins for a 620 x 480 detector (Table 2) and the
    91 / 725 / 1381 bins of the 64^2 / 512^2 / 976^2 detectors used here."""
    return int(math.ceil(math.sqrt(nu * nu + nv * nv)))


@dataclass
class Views:
    """Per-view frames, float64 arrays of shape [V, 3]."""
    src: np.ndarray
    det_center: np.ndarray
    ex: np.ndarray
    ey: np.ndarray
    tangent: np.ndarray
    meta: dict = field(default_factory=dict)

    def __len__(self):
        return self.src.shape[0]

    def subset(self, idx):
        idx = np.asarray(idx)
        return Views(self.src[idx].copy(), self.det_center[idx].copy(),
                     self.ex[idx].copy(), self.ey[idx].copy(),
                     self.tangent[idx].copy(), dict(self.meta, subset=idx.tolist()))

    def packed(self) -> np.ndarray:
        """[V, 15] float64: src, det_center, ex, ey, tangent (C-ABI dc_view order)."""
        return np.ascontiguousarray(np.concatenate(
            [self.src, self.det_center, self.ex, self.ey, self.tangent], axis=1))

    @staticmethod
    def concat(parts, meta=None):
        return Views(*(np.concatenate([getattr(p, k) for p in parts], axis=0)
                       for k in ("src", "det_center", "ex", "ey", "tangent")),
                     meta=meta or {})


def _sphere_frames(theta, phi, dtheta, dphi, sid, sdd):
    """Source on the sphere of radius sid, detector opposite, facing the centre.

    theta/phi are azimuth/elevation per view; dtheta/dphi are the per-view
    increments of the orbit parameter (used to form t = a' dlambda)."""
    theta = np.asarray(theta, np.float64)
    phi = np.asarray(phi, np.float64)
    ct, st, cp, sp = np.cos(theta), np.sin(theta), np.cos(phi), np.sin(phi)
    src = sid * np.stack([cp * ct, cp * st, sp], axis=1)
    lz = src / sid
    ex = np.stack([-st, ct, np.zeros_like(st)], axis=1)
    ey = np.cross(lz, ex)
    ey /= np.linalg.norm(ey, axis=1, keepdims=True)
    det = src - sdd * lz
    da_dtheta = sid * np.stack([-cp * st, cp * ct, np.zeros_like(st)], axis=1)
    da_dphi = sid * np.stack([-sp * ct, -sp * st, cp], axis=1)
    tangent = da_dtheta * np.asarray(dtheta)[:, None] + da_dphi * np.asarray(dphi)[:, None]
    return src, det, ex, ey, tangent


def circle_orbit(n_views, sid, sdd, start=0.0, span=2 * math.pi):
    """Circular orbit in the plane z = 0 (paper, Sec. 4.1)."""
    lam = start + np.arange(n_views) * (span / n_views)
    d = np.full(n_views, span / n_views)
    src, det, ex, ey, t = _sphere_frames(lam, np.zeros(n_views), d, np.zeros(n_views), sid, sdd)
    meta = {"kind": "circle", "sid": sid, "sdd": sdd,
            "segments": [{"kind": "circle", "start": 0, "count": n_views, "closed": span >= 2 * math.pi - 1e-12,
                          "lam0": start, "dlam": span / n_views}]}
    return Views(src, det, ex, ey, t, meta)


def sinusoid_orbit(n_views, sid, sdd, amp_mm=100.0, periods=2, phi_max=None):
    """Sinusoidal orbit on the sphere (paper, eq. 15): phi = phi_max cos(f theta),
    theta uniform over [-pi, pi).  phi_max defaults to asin(amp_mm / sid)."""
    if phi_max is None:
        phi_max = math.asin(amp_mm / sid)
    dth = 2 * math.pi / n_views
    th = -math.pi + np.arange(n_views) * dth
    phi = phi_max * np.cos(periods * th)
    dphi = -phi_max * periods * np.sin(periods * th) * dth
    src, det, ex, ey, t = _sphere_frames(th, phi, np.full(n_views, dth), dphi, sid, sdd)
    meta = {"kind": "sinusoid", "sid": sid, "sdd": sdd,
            "segments": [{"kind": "sinusoid", "start": 0, "count": n_views, "closed": True,
                          "phi_max": phi_max, "freq": periods, "th0": -math.pi, "dth": dth}]}
    return Views(src, det, ex, ey, t, meta)


def circle_arc_orbit(n_arc, n_circ, sid, sdd, tilt_deg=30.0):
    """Circle plus an orthogonal arc (paper, Sec. 4.3).  Arc views come first
    (elevation from -tilt to +tilt at azimuth 0, endpoints included), then the
    full circle."""
    tilt = math.radians(tilt_deg)
    dphi = 2 * tilt / (n_arc - 1)
    phi = -tilt + np.arange(n_arc) * dphi
    arc = _sphere_frames(np.zeros(n_arc), phi, np.zeros(n_arc), np.full(n_arc, dphi), sid, sdd)
    dl = 2 * math.pi / n_circ
    lam = np.arange(n_circ) * dl
    circ = _sphere_frames(lam, np.zeros(n_circ), np.full(n_circ, dl), np.zeros(n_circ), sid, sdd)
    parts = [Views(*arc), Views(*circ)]
    meta = {"kind": "circle_arc", "sid": sid, "sdd": sdd,
            "segments": [{"kind": "arc", "start": 0, "count": n_arc, "closed": False,
                          "phi0": -tilt, "dphi": dphi},
                         {"kind": "circle", "start": n_arc, "count": n_circ, "closed": True,
                          "lam0": 0.0, "dlam": dl}]}
    return Views.concat(parts, meta)


def circle_line_orbit(n_circ, n_line, sid, sdd, half_len):
    """Circle in z = 0 plus a line parallel to z through (sid, 0, 0); along the
    line the detector keeps the orientation of the circle view at azimuth 0."""
    circ = circle_orbit(n_circ, sid, sdd)
    dz = 2 * half_len / (n_line - 1)
    z = -half_len + np.arange(n_line) * dz
    src = np.stack([np.full(n_line, sid), np.zeros(n_line), z], axis=1)
    lz = np.tile([1.0, 0.0, 0.0], (n_line, 1))
    ex = np.tile([0.0, 1.0, 0.0], (n_line, 1))
    ey = np.cross(lz, ex)
    det = src - sdd * lz
    t = np.tile([0.0, 0.0, dz], (n_line, 1))
    line = Views(src, det, ex, ey, t)
    meta = {"kind": "circle_line", "sid": sid, "sdd": sdd,
            "segments": [dict(circ.meta["segments"][0]),
                         {"kind": "line", "start": n_circ, "count": n_line, "closed": False,
                          "z0": -half_len, "dz": dz}]}
    return Views.concat([circ, line], meta)


def random_nn_orbit(n_views, sid, sdd, tilt_deg=10.0, seed=0):
    """Random nearest-neighbour orbit (paper, Sec. 4.4): azimuth U[0, 2pi),
    elevation U[-tilt, tilt], reordered greedily by nearest neighbour from the
    first point; tangent by central differences of the source positions."""
    rng = np.random.Generator(np.random.PCG64(seed))
    th = rng.uniform(0, 2 * math.pi, n_views)
    ph = rng.uniform(-math.radians(tilt_deg), math.radians(tilt_deg), n_views)
    pts = sid * np.stack([np.cos(ph) * np.cos(th), np.cos(ph) * np.sin(th), np.sin(ph)], 1)
    order = [0]
    left = set(range(1, n_views))
    while left:
        cur = pts[order[-1]]
        cand = np.fromiter(left, dtype=np.int64)
        nxt = int(cand[np.argmin(np.linalg.norm(pts[cand] - cur, axis=1))])
        order.append(nxt)
        left.remove(nxt)
    th, ph = th[order], ph[order]
    src, det, ex, ey, _ = _sphere_frames(th, ph, np.zeros(n_views), np.zeros(n_views), sid, sdd)
    t = np.empty_like(src)
    t[1:-1] = 0.5 * (src[2:] - src[:-2])
    t[0] = src[1] - src[0]
    t[-1] = src[-1] - src[-2]
    meta = {"kind": "random_nn", "sid": sid, "sdd": sdd,
            "segments": [{"kind": "samples", "start": 0, "count": n_views, "closed": False}]}
    return Views(src, det, ex, ey, t, meta)


# ---------------------------------------------------------------------------
# Workloads.  C1..C5 are the five scan configurations the library is measured
# and parity-tested on; paper_geometry() below is the paper's own (Tables 1 and 2).
# ---------------------------------------------------------------------------
CONFIGS = {
    "C1": dict(orbit="circle", n_views=90, vol=32, vox=1.0, det=64, pitch=1.0, n_theta=180,
               sid=750.0, sdd=1200.0, n_ell=5, seed=1, noise=None),
    "C2": dict(orbit="sinusoid", n_views=496, vol=256, vox=0.5, det=512, pitch=0.6, n_theta=360,
               sid=750.0, sdd=1200.0, n_ell=20, seed=2, noise=1e5, amp_mm=100.0, periods=2),
    "C3": dict(orbit="circle_arc", n_views=460, n_arc=100, n_circ=360, tilt=30.0, vol=256, vox=0.5,
               det=512, pitch=0.6, n_theta=360, sid=750.0, sdd=1200.0, n_ell=20, seed=3, noise=None),
    "C5": dict(orbit="sinusoid", n_views=496, vol=512, vox=0.25, det=976, pitch=0.308, n_theta=720,
               sid=750.0, sdd=1200.0, n_ell=20, seed=5, noise=None, amp_mm=100.0, periods=2),
}


def config_geometry(name: str, n_views: int | None = None):
    """(Grid, Views) for a named workload.  n_views overrides the orbit
    sampling density (used for small parity cases)."""
    c = CONFIGS[name]
    nu = nv = c["det"]
    grid = Grid(nu=nu, nv=nv, du=c["pitch"], dv=c["pitch"], n_theta=c["n_theta"],
                n_s=radon_bins(nu, nv), ds=c["pitch"], nx=c["vol"], ny=c["vol"], nz=c["vol"],
                vx=c["vox"], vy=c["vox"], vz=c["vox"])
    nvw = n_views or c["n_views"]
    if c["orbit"] == "circle":
        views = circle_orbit(nvw, c["sid"], c["sdd"])
    elif c["orbit"] == "sinusoid":
        views = sinusoid_orbit(nvw, c["sid"], c["sdd"], c["amp_mm"], c["periods"])
    elif c["orbit"] == "circle_arc":
        if n_views is None:
            views = circle_arc_orbit(c["n_arc"], c["n_circ"], c["sid"], c["sdd"], c["tilt"])
        else:
            na = max(2, round(n_views * c["n_arc"] / c["n_views"]))
            views = circle_arc_orbit(na, n_views - na, c["sid"], c["sdd"], c["tilt"])
    else:
        raise ValueError(c["orbit"])
    return grid, views


def paper_geometry():
    """The paper's reconstruction geometry (its Tables 1 and 2 and the sinusoidal
    orbit section): a 128 x 512 x 512 volume (z, y, x) of 0.25 mm voxels, 400 views
    of a 620 x 480 detector with 0.616 mm pixels, SID 750 mm, SDD 1200 mm, the
    sinusoid with a 20 degree maximum tilt and frequency 5, and a Radon grid of 360
    angles by 785 bins of 0.616 mm."""
    grid = Grid(nu=620, nv=480, du=0.616, dv=0.616, n_theta=360, n_s=radon_bins(620, 480), ds=0.616,
                nx=512, ny=512, nz=128, vx=0.25, vy=0.25, vz=0.25)
    views = sinusoid_orbit(400, 750.0, 1200.0, phi_max=math.radians(20.0), periods=5)
    return grid, views


# Batched training workload: 8 scans on the C2 grid with mixed orbits and view
# counts from 248 to 496 (3002 views), one phantom seed each.
C4_MIX = [("circle", 248), ("sinusoid", 496), ("circle_arc", (100, 360)), ("circle", 496),
          ("sinusoid", 248), ("circle_arc", (60, 250)), ("circle", 372), ("sinusoid", 372)]
C4_SEEDS = list(range(40, 48))


def c4_scans():
    """(Grid, [Views per scan], [phantom seed per scan]) of the batched workload."""
    c = CONFIGS["C2"]
    grid, _ = config_geometry("C2", n_views=4)
    sets = []
    for kind, n in C4_MIX:
        if kind == "circle":
            sets.append(circle_orbit(n, c["sid"], c["sdd"]))
        elif kind == "sinusoid":
            sets.append(sinusoid_orbit(n, c["sid"], c["sdd"], c["amp_mm"], c["periods"]))
        else:
            sets.append(circle_arc_orbit(n[0], n[1], c["sid"], c["sdd"], 30.0))
    return grid, sets, list(C4_SEEDS)
