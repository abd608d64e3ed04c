"""Smooth Crofton redundancy weight M(theta, lambda) of eq. 9, float64.

    M(theta, lambda) = |a'(lambda).theta|^m c(lambda) / sum_alpha |a'(lambda_alpha).theta|^m c(lambda_alpha)

where lambda_alpha runs over every orbit parameter whose source position lies
in the plane through a(lambda) with normal theta (Defrise & Clack's smooth
replacement of 1/n(theta, lambda), Sec. 2.4).  Readings: m = 2; a' is the
tangent per view step (a' dlambda, so segments sampled differently are weighted
by their per-view displacement); c = 1 on closed segments and a raised-cosine
taper over the last 5 % of each end of an open segment, floored at 0.01 so it
stays positive; where every term vanishes (a plane tangent to the orbit at all
its intersections) M = 1/n.

Orbits are taken from the analytic segment descriptions attached to the view
list (circle, arc, line, sinusoid).  Intersections are solved in closed form
on circles, arcs and lines, and by dense sign-change search plus bisection on
the sinusoid.
"""
from __future__ import annotations

import math

import numpy as np

M_EXP = 2
TAPER = 0.05
C_FLOOR = 0.01
DEGENERATE = 1e-18   # relative size below which every |a'.theta|^m term is taken as zero


class Orbit:
    def __init__(self, views):
        self.sid = float(views.meta["sid"])
        self.segs = views.meta["segments"]

    # ---- per-segment parameterisation: view k of segment -> parameter tau
    def tau_of_view(self, seg, k):
        s = self.segs[seg]
        if s["kind"] == "circle":
            return s["lam0"] + k * s["dlam"]
        if s["kind"] == "arc":
            return s["phi0"] + k * s["dphi"]
        if s["kind"] == "line":
            return s["z0"] + k * s["dz"]
        if s["kind"] == "sinusoid":
            return s["th0"] + k * s["dth"]
        raise ValueError(s["kind"])

    def locate(self, v):
        for i, s in enumerate(self.segs):
            if s["start"] <= v < s["start"] + s["count"]:
                return i, self.tau_of_view(i, v - s["start"])
        raise IndexError(v)

    def point(self, seg, tau):
        s, R = self.segs[seg], self.sid
        tau = np.asarray(tau, np.float64)
        if s["kind"] == "circle":
            return np.stack([R * np.cos(tau), R * np.sin(tau), 0 * tau], -1)
        if s["kind"] == "arc":
            return np.stack([R * np.cos(tau), 0 * tau, R * np.sin(tau)], -1)
        if s["kind"] == "line":
            return np.stack([R + 0 * tau, 0 * tau, tau], -1)
        if s["kind"] == "sinusoid":
            ph = s["phi_max"] * np.cos(s["freq"] * tau)
            return R * np.stack([np.cos(ph) * np.cos(tau), np.cos(ph) * np.sin(tau), np.sin(ph)], -1)
        raise ValueError(s["kind"])

    def tangent(self, seg, tau):
        """a'(tau) times the segment's per-view parameter step."""
        s, R = self.segs[seg], self.sid
        tau = np.asarray(tau, np.float64)
        if s["kind"] == "circle":
            return s["dlam"] * np.stack([-R * np.sin(tau), R * np.cos(tau), 0 * tau], -1)
        if s["kind"] == "arc":
            return s["dphi"] * np.stack([-R * np.sin(tau), 0 * tau, R * np.cos(tau)], -1)
        if s["kind"] == "line":
            return np.stack([0 * tau, 0 * tau, s["dz"] + 0 * tau], -1)
        if s["kind"] == "sinusoid":
            f, pm = s["freq"], s["phi_max"]
            ph = pm * np.cos(f * tau)
            dph = -pm * f * np.sin(f * tau)
            da = R * np.stack([-np.sin(ph) * dph * np.cos(tau) - np.cos(ph) * np.sin(tau),
                               -np.sin(ph) * dph * np.sin(tau) + np.cos(ph) * np.cos(tau),
                               np.cos(ph) * dph], -1)
            return s["dth"] * da
        raise ValueError(s["kind"])

    def taper(self, seg, tau):
        s = self.segs[seg]
        if s["closed"]:
            return np.ones_like(np.asarray(tau, np.float64))
        t0 = self.tau_of_view(seg, 0)
        t1 = self.tau_of_view(seg, s["count"] - 1)
        u = (np.asarray(tau, np.float64) - t0) / (t1 - t0)
        e = np.minimum(u, 1.0 - u) / TAPER
        ramp = np.where(e < 1.0, 0.5 - 0.5 * np.cos(math.pi * np.clip(e, 0, 1)), 1.0)
        return C_FLOOR + (1.0 - C_FLOOR) * ramp

    # ---- all parameters on segment `seg` whose point lies in {p : p.theta = d}
    def roots(self, seg, theta, d, fine=64):
        s, R = self.segs[seg], self.sid
        th = np.asarray(theta, np.float64)
        if s["kind"] in ("circle", "arc"):
            c1 = th[0]
            c2 = th[1] if s["kind"] == "circle" else th[2]
            rho = R * math.hypot(c1, c2)
            if rho == 0.0 or abs(d) > rho * (1 + 1e-12):
                return []
            base = math.atan2(c2, c1)
            ac = math.acos(max(-1.0, min(1.0, d / rho)))
            cand = [base + ac, base - ac] if ac > 0 else [base]
            if s["kind"] == "circle":
                if s["closed"]:
                    return [float(np.mod(c - s["lam0"], 2 * math.pi) + s["lam0"]) for c in cand]
                # an open circle only holds the parameters its views cover; the
                # window starts 1e-12 below the first view's parameter, so that a
                # crossing at the first source point survives rounding (as on arcs)
                lo, hi = self.tau_of_view(seg, 0), self.tau_of_view(seg, s["count"] - 1)
                taus = [float(np.mod(c - lo + 1e-12, 2 * math.pi) + lo - 1e-12) for c in cand]
                return [min(max(t, lo), hi) for t in taus if t <= hi + 1e-12]
            lo, hi = self.tau_of_view(seg, 0), self.tau_of_view(seg, s["count"] - 1)
            out = []
            for c in cand:
                c = (c + math.pi) % (2 * math.pi) - math.pi
                if lo - 1e-12 <= c <= hi + 1e-12:
                    out.append(min(max(c, lo), hi))
            return out
        if s["kind"] == "line":
            if th[2] == 0.0:
                return []
            z = (d - R * th[0]) / th[2]
            lo, hi = self.tau_of_view(seg, 0), self.tau_of_view(seg, s["count"] - 1)
            return [z] if lo - 1e-12 <= z <= hi + 1e-12 else []
        if s["kind"] == "sinusoid":
            n = fine * s["count"]
            tau = s["th0"] + (np.arange(n) + 0.5) * (2 * math.pi / n)
            F = self.point(seg, tau) @ th - d
            out = []
            for j in np.nonzero(np.sign(F[:-1]) * np.sign(F[1:]) <= 0)[0]:
                a, b = tau[j], tau[j + 1]
                fa = F[j]
                for _ in range(80):
                    mid = 0.5 * (a + b)
                    fm = float(self.point(seg, mid) @ th - d)
                    if (fm <= 0) == (fa <= 0):
                        a, fa = mid, fm
                    else:
                        b = mid
                out.append(0.5 * (a + b))
            # the wrap-around interval
            if np.sign(F[-1]) * np.sign(F[0]) < 0:
                a, b, fa = tau[-1], tau[0] + 2 * math.pi, F[-1]
                for _ in range(80):
                    mid = 0.5 * (a + b)
                    fm = float(self.point(seg, mid) @ th - d)
                    if (fm <= 0) == (fa <= 0):
                        a, fa = mid, fm
                    else:
                        b = mid
                out.append(0.5 * (a + b))
            return out
        raise ValueError(s["kind"])

    def intersections(self, theta, d):
        return [(seg, r) for seg in range(len(self.segs)) for r in self.roots(seg, theta, d)]

    def weight_at(self, seg, tau, theta):
        return abs(float(self.tangent(seg, tau) @ theta)) ** M_EXP * float(self.taper(seg, tau))


def M_point(orbit: Orbit, seg, tau, theta):
    """Eq. 9 at orbit point (seg, tau) for the plane with unit normal theta through it."""
    theta = np.asarray(theta, np.float64)
    d = float(orbit.point(seg, tau) @ theta)
    hits = orbit.intersections(theta, d)
    den = sum(orbit.weight_at(s, r, theta) for s, r in hits)
    if den <= DEGENERATE * float(np.linalg.norm(orbit.tangent(seg, tau))) ** M_EXP:
        return 1.0 / max(1, len(hits))
    return orbit.weight_at(seg, tau, theta) / den


def M_view(views, grid, v, bins=None):
    """M[k][m] of view v on the Radon grid; theta_km = (D n_mu + s l_z)/sqrt(s^2+D^2).

    ``bins`` optionally restricts to a list of (k, m) pairs (returns a vector)."""
    orbit = Orbit(views)
    seg, tau = orbit.locate(v)
    lx, ly = np.asarray(views.ex[v]), np.asarray(views.ey[v])
    lz = np.cross(lx, ly)
    D = float(np.dot(views.src[v] - views.det_center[v], lz))
    mu = np.arange(grid.n_theta) * math.pi / grid.n_theta
    s = (np.arange(grid.n_s) - (grid.n_s - 1) / 2.0) * grid.ds
    todo = bins if bins is not None else [(k, m) for k in range(grid.n_theta) for m in range(grid.n_s)]
    out = []
    for k, m in todo:
        n = math.cos(mu[k]) * lx + math.sin(mu[k]) * ly
        th = (D * n + s[m] * lz) / math.hypot(s[m], D)
        out.append(M_point(orbit, seg, tau, th))
    out = np.asarray(out)
    return out if bins is not None else out.reshape(grid.n_theta, grid.n_s)


def M_view_closed_form(views, grid, v):
    """Vectorised M[k][m] of view v for orbits made only of circles, arcs and
    lines, where every plane-orbit intersection has a closed form."""
    orbit = Orbit(views)
    R = orbit.sid
    seg_v, tau_v = orbit.locate(v)
    lx, ly = np.asarray(views.ex[v]), np.asarray(views.ey[v])
    lz = np.cross(lx, ly)
    a_v = np.asarray(views.src[v], np.float64)
    D = float(np.dot(a_v - views.det_center[v], lz))
    mu = np.arange(grid.n_theta) * math.pi / grid.n_theta
    s = (np.arange(grid.n_s) - (grid.n_s - 1) / 2.0) * grid.ds
    n = np.cos(mu)[:, None, None] * lx + np.sin(mu)[:, None, None] * ly          # [K,1,3]
    th = (D * n + s[None, :, None] * lz) / np.hypot(s, D)[None, :, None]         # [K,M,3]
    d = th @ a_v
    den = np.zeros(d.shape)
    count = np.zeros(d.shape)

    def add(seg, tau, ok):
        w = np.abs(np.einsum("...i,...i->...", orbit.tangent(seg, np.where(ok, tau, 0.0)), th)) ** M_EXP
        w = w * orbit.taper(seg, np.where(ok, tau, orbit.tau_of_view(seg, 0)))
        return np.where(ok, w, 0.0), ok.astype(float)

    for seg, sd in enumerate(orbit.segs):
        if sd["kind"] in ("circle", "arc"):
            c1 = th[..., 0]
            c2 = th[..., 1] if sd["kind"] == "circle" else th[..., 2]
            rho = R * np.hypot(c1, c2)
            with np.errstate(divide="ignore", invalid="ignore"):
                ratio = np.where(rho > 0, d / rho, 2.0)
            hit = np.abs(ratio) <= 1.0 + 1e-12
            base = np.arctan2(c2, c1)
            ac = np.arccos(np.clip(ratio, -1, 1))
            for sign in (1.0, -1.0):
                tau = base + sign * ac
                if sd["kind"] == "circle":
                    ok = hit & ((sign > 0) | (ac > 0))
                    if not sd["closed"]:
                        lo, hi = orbit.tau_of_view(seg, 0), orbit.tau_of_view(seg, sd["count"] - 1)
                        tau = np.mod(tau - lo + 1e-12, 2 * math.pi) + lo - 1e-12
                        ok = ok & (tau <= hi + 1e-12)
                        tau = np.clip(tau, lo, hi)
                else:
                    tau = np.mod(tau + math.pi, 2 * math.pi) - math.pi
                    lo, hi = orbit.tau_of_view(seg, 0), orbit.tau_of_view(seg, sd["count"] - 1)
                    ok = hit & ((sign > 0) | (ac > 0)) & (tau >= lo - 1e-12) & (tau <= hi + 1e-12)
                    tau = np.clip(tau, lo, hi)
                w, c = add(seg, tau, ok)
                den += w
                count += c
        elif sd["kind"] == "line":
            with np.errstate(divide="ignore", invalid="ignore"):
                z = (d - R * th[..., 0]) / th[..., 2]
            lo, hi = orbit.tau_of_view(seg, 0), orbit.tau_of_view(seg, sd["count"] - 1)
            ok = np.isfinite(z) & (z >= lo - 1e-12) & (z <= hi + 1e-12)
            w, c = add(seg, np.clip(np.nan_to_num(z), lo, hi), ok)
            den += w
            count += c
        else:
            raise ValueError("closed form needs circle/arc/line segments, got " + sd["kind"])
    t_v = orbit.tangent(seg_v, tau_v)
    num = np.abs(th @ t_v) ** M_EXP * float(orbit.taper(seg_v, tau_v))
    tol = DEGENERATE * float(np.linalg.norm(t_v)) ** M_EXP
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(den > tol, num / den, 1.0 / np.maximum(count, 1.0))
