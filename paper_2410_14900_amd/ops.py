"""Torch-facing binding of the C ABI: same names as include/dcfbp.h.

Only argument marshalling happens here: shapes and dtypes are checked, torch
tensors are turned into device pointers, and the call is enqueued on torch's
current stream.  Every arithmetic step runs in the HIP library.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import DcGrid, DcView, check

_DT = {torch.float32: _lib.DC_F32, torch.bfloat16: _lib.DC_BF16, torch.float16: _lib.DC_F16}
MODES = {"analytic": _lib.DC_WEIGHT_ANALYTIC, "raw": _lib.DC_WEIGHT_RAW}


def make_grid(grid) -> DcGrid:
    d = grid if isinstance(grid, dict) else grid.__dict__
    return DcGrid(**{k: d[k] for k, _ in DcGrid._fields_})


def make_views(views):
    arr = views.packed() if hasattr(views, "packed") else np.asarray(views, np.float64)
    arr = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1, 15)
    buf = (DcView * arr.shape[0])()
    ctypes.memmove(buf, arr.ctypes.data, arr.nbytes)
    return buf, arr.shape[0]


def validate(grid, views):
    """Host-only geometry check; returns (status, message)."""
    g = make_grid(grid)
    buf, n = make_views(views)
    st = _lib.lib().dc_validate(ctypes.byref(g), buf, n)
    return st, (_lib.last_error() if st else "")


def plan_bounds(grid, views):
    """Host-only bounds and kernel forms of a one-scan plan (dc_plan_bounds), as a dict."""
    g = make_grid(grid)
    buf, n = make_views(views)
    b = _lib.DcBounds()
    check(_lib.lib().dc_plan_bounds(ctypes.byref(g), buf, n, ctypes.byref(b)), "dc_plan_bounds")
    out = {name: getattr(b, name) for name, _ in _lib.DcBounds._fields_}
    out["bp_block"] = tuple(b.bp_block)
    out["interp_tile"] = tuple(b.interp_tile)
    return out


class Plan:
    """Geometry plan on the current device (small float64-derived tables).

    With ``first_view`` (n_samples + 1 increasing view indices) the plan is
    batched: several scans sharing the grid, views back to back, and volumes of
    shape (n_samples, nz, ny, nx).  ``Plan.batched(grid, [views, ...])`` builds one
    from a list of per-scan view sets."""

    def __init__(self, grid, views, first_view=None):
        self.grid = make_grid(grid)
        buf, n = make_views(views)
        h = ctypes.c_void_p()
        L = _lib.lib()
        if first_view is None:
            check(L.dc_plan_create(ctypes.byref(self.grid), buf, n, 0, ctypes.byref(h)), "dc_plan_create")
        else:
            fv = [int(x) for x in first_view]
            arr = (ctypes.c_int32 * len(fv))(*fv)
            check(L.dc_plan_create_batched(ctypes.byref(self.grid), buf, n, arr, len(fv) - 1, 0, ctypes.byref(h)),
                  "dc_plan_create_batched")
        self.handle = h
        self.n_views = n
        self.n_samples = L.dc_plan_n_samples(h)
        self.first_view = [0, n] if first_view is None else [int(x) for x in first_view]
        g = self.grid
        self.det_shape = (g.nv, g.nu)
        self.sino_shape = (g.n_theta, g.n_s)
        self.vol_shape = (g.nz, g.ny, g.nx) if first_view is None else (self.n_samples, g.nz, g.ny, g.nx)

    @classmethod
    def batched(cls, grid, view_sets):
        """One plan over several scans (each a view set with ``packed()`` or an [n][15] array)."""
        parts = [np.ascontiguousarray(v.packed() if hasattr(v, "packed") else v, np.float64).reshape(-1, 15)
                 for v in view_sets]
        first = np.concatenate([[0], np.cumsum([len(p) for p in parts])])
        return cls(grid, np.concatenate(parts), first_view=first)

    KNOB_NAMES = ("splat_angles", "interp_tile_u", "interp_angles", "bp_block_y", "fp_tile_u")

    def knobs(self):
        """The kernels' work shapes (dc_plan_get_knobs) as a dict."""
        k = _lib.DcKnobs()
        check(_lib.lib().dc_plan_get_knobs(self.handle, ctypes.byref(k)), "dc_plan_get_knobs")
        return {n: getattr(k, n) for n in self.KNOB_NAMES}

    def set_knobs(self, **values):
        """Sets some knobs (dc_plan_set_knobs); the others keep their values."""
        cur = self.knobs()
        unknown = set(values) - set(cur)
        if unknown:
            raise ValueError("unknown knobs: %s" % sorted(unknown))
        cur.update(values)
        k = _lib.DcKnobs(**{n: int(cur[n]) for n in self.KNOB_NAMES})
        check(_lib.lib().dc_plan_set_knobs(self.handle, ctypes.byref(k)), "dc_plan_set_knobs")
        return self.knobs()

    def autotune(self, stream=None):
        """Times the knob candidates on this plan's geometry and keeps the fastest
        (dc_plan_autotune; DCFBP_KNOBS and DCFBP_TUNE_CACHE apply).  Returns
        {"knobs": ..., "ms": {stage: ms}, "source": "timed" | "cache" | "environment"}."""
        k = _lib.DcKnobs()
        ms = (ctypes.c_double * 4)()
        src = ctypes.c_int32()
        check(_lib.lib().dc_plan_autotune(self.handle, 0, _stream(stream), ctypes.byref(k), ms, ctypes.byref(src)),
              "dc_plan_autotune")
        return {"knobs": {n: getattr(k, n) for n in self.KNOB_NAMES},
                "ms": dict(zip(("weight_radon", "detector_bp", "cone_bp", "cone_bp_adjoint"), list(ms))),
                "source": ("timed", "cache", "environment")[src.value]}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.lib().dc_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, name, shape, dtypes=(torch.float32,), nullable=False):
    if t is None:
        if nullable:
            return
        raise ValueError("%s is required" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if t.dtype not in dtypes:
        raise ValueError("%s has dtype %s, expected one of %s" % (name, t.dtype, dtypes))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _range(plan, v0, nv):
    if nv is None:
        nv = plan.n_views - v0
    return int(v0), int(nv)


ANY = tuple(_DT)


def dc_weight_radon(plan, g, R, v0=0, nv=None, stream=None):
    V = plan.n_views
    _need(g, "g", (V,) + plan.det_shape)
    _need(R, "R", (V,) + plan.sino_shape, ANY)
    v0, nv = _range(plan, v0, nv)
    check(_lib.lib().dc_weight_radon(plan.handle, _ptr(g), _ptr(R), _DT[R.dtype], v0, nv, _stream(stream)),
          "dc_weight_radon")
    return R


def dc_weight_radon_noalloc(plan, g, R, v0=0, nv=None, stream=None):
    """dc_weight_radon with its scratch in the library's static device array
    (allocates nothing; calls on one GPU must not overlap)."""
    V = plan.n_views
    _need(g, "g", (V,) + plan.det_shape)
    _need(R, "R", (V,) + plan.sino_shape, ANY)
    v0, nv = _range(plan, v0, nv)
    check(_lib.lib().dc_weight_radon_noalloc(plan.handle, _ptr(g), _ptr(R), _DT[R.dtype], v0, nv,
                                             _stream(stream)), "dc_weight_radon_noalloc")
    return R


def dc_weight_radon_adjoint(plan, GR, Gg, v0=0, nv=None, stream=None):
    V = plan.n_views
    _need(GR, "GR", (V,) + plan.sino_shape, ANY)
    _need(Gg, "Gg", (V,) + plan.det_shape)
    v0, nv = _range(plan, v0, nv)
    check(_lib.lib().dc_weight_radon_adjoint(plan.handle, _ptr(GR), _DT[GR.dtype], _ptr(Gg), v0, nv,
                                             _stream(stream)), "dc_weight_radon_adjoint")
    return Gg


def dc_filter(plan, R, M, H, mode="analytic", v0=0, nv=None, stream=None):
    V = plan.n_views
    _need(R, "R", (V,) + plan.sino_shape, ANY)
    _need(M, "M", (V,) + plan.sino_shape)
    _need(H, "H", (V,) + plan.sino_shape, ANY)
    v0, nv = _range(plan, v0, nv)
    check(_lib.lib().dc_filter(plan.handle, _ptr(R), _DT[R.dtype], _ptr(M), MODES[mode], _ptr(H), _DT[H.dtype],
                               v0, nv, _stream(stream)), "dc_filter")
    return H


def dc_filter_adjoint(plan, GH, R, M, GM=None, GR=None, mode="analytic", accumulate_GM=False, v0=0, nv=None,
                      stream=None):
    V = plan.n_views
    _need(GH, "GH", (V,) + plan.sino_shape, ANY)
    _need(R, "R", (V,) + plan.sino_shape, ANY)
    _need(M, "M", (V,) + plan.sino_shape)
    _need(GM, "GM", (V,) + plan.sino_shape, nullable=True)
    _need(GR, "GR", (V,) + plan.sino_shape, nullable=True)
    v0, nv = _range(plan, v0, nv)
    check(_lib.lib().dc_filter_adjoint(plan.handle, _ptr(GH), _DT[GH.dtype], _ptr(R), _DT[R.dtype], _ptr(M),
                                       MODES[mode], _ptr(GM), int(bool(accumulate_GM)), _ptr(GR), v0, nv,
                                       _stream(stream)), "dc_filter_adjoint")
    return GM, GR


def dc_detector_bp(plan, H, gF, v0=0, nv=None, stream=None):
    V = plan.n_views
    _need(H, "H", (V,) + plan.sino_shape, ANY)
    _need(gF, "gF", (V,) + plan.det_shape, ANY)
    v0, nv = _range(plan, v0, nv)
    check(_lib.lib().dc_detector_bp(plan.handle, _ptr(H), _DT[H.dtype], _ptr(gF), _DT[gF.dtype], v0, nv,
                                    _stream(stream)), "dc_detector_bp")
    return gF


def dc_detector_bp_adjoint(plan, GgF, GH, v0=0, nv=None, stream=None):
    V = plan.n_views
    _need(GgF, "GgF", (V,) + plan.det_shape, ANY)
    _need(GH, "GH", (V,) + plan.sino_shape, ANY)
    v0, nv = _range(plan, v0, nv)
    check(_lib.lib().dc_detector_bp_adjoint(plan.handle, _ptr(GgF), _DT[GgF.dtype], _ptr(GH), _DT[GH.dtype], v0,
                                            nv, _stream(stream)), "dc_detector_bp_adjoint")
    return GH


def dc_cone_bp(plan, gF, f, accumulate=False, relu=False, v0=0, nv=None, stream=None):
    V = plan.n_views
    _need(gF, "gF", (V,) + plan.det_shape, ANY)
    _need(f, "f", plan.vol_shape)
    v0, nv = _range(plan, v0, nv)
    check(_lib.lib().dc_cone_bp(plan.handle, _ptr(gF), _DT[gF.dtype], _ptr(f), int(bool(accumulate)),
                                int(bool(relu)), v0, nv, _stream(stream)), "dc_cone_bp")
    return f


def dc_cone_bp_adjoint(plan, Gf, GgF, f_relu=None, v0=0, nv=None, stream=None):
    V = plan.n_views
    _need(Gf, "Gf", plan.vol_shape)
    _need(f_relu, "f_relu", plan.vol_shape, nullable=True)
    _need(GgF, "GgF", (V,) + plan.det_shape, ANY)
    v0, nv = _range(plan, v0, nv)
    check(_lib.lib().dc_cone_bp_adjoint(plan.handle, _ptr(Gf), _ptr(f_relu), _ptr(GgF), _DT[GgF.dtype], v0, nv,
                                        _stream(stream)), "dc_cone_bp_adjoint")
    return GgF


def dc_smooth_weights(plan, M, Ms, sigma=20.0, radius=60, v0=0, nv=None, stream=None):
    """Gaussian filter layer on the weight (Ms may be M itself)."""
    V = plan.n_views
    _need(M, "M", (V,) + plan.sino_shape)
    _need(Ms, "Ms", (V,) + plan.sino_shape)
    v0, nv = _range(plan, v0, nv)
    check(_lib.lib().dc_smooth_weights(plan.handle, _ptr(M), _ptr(Ms), float(sigma), int(radius), v0, nv,
                                       _stream(stream)), "dc_smooth_weights")
    return Ms


def dc_smooth_weights_adjoint(plan, GMs, GM, sigma=20.0, radius=60, v0=0, nv=None, stream=None):
    """Transpose of dc_smooth_weights (GM may be GMs itself)."""
    V = plan.n_views
    _need(GMs, "GMs", (V,) + plan.sino_shape)
    _need(GM, "GM", (V,) + plan.sino_shape)
    v0, nv = _range(plan, v0, nv)
    check(_lib.lib().dc_smooth_weights_adjoint(plan.handle, _ptr(GMs), _ptr(GM), float(sigma), int(radius), v0,
                                               nv, _stream(stream)), "dc_smooth_weights_adjoint")
    return GM


_SEG_KINDS = {"circle": _lib.DC_SEG_CIRCLE, "arc": _lib.DC_SEG_ARC, "line": _lib.DC_SEG_LINE,
              "sinusoid": _lib.DC_SEG_SINUSOID}
_SEG_PARAMS = {"circle": ("lam0", "dlam"), "arc": ("phi0", "dphi"), "line": ("z0", "dz"), "sinusoid": ("th0", "dth")}


def make_segments(segments):
    """ctypes array of dc_orbit_segment from analytic segment descriptions (dicts
    with kind, start, count, closed and the kind's parameters, as synth's orbits
    carry them in views.meta["segments"])."""
    buf = (_lib.DcOrbitSegment * len(segments))()
    for i, s in enumerate(segments):
        if s["kind"] not in _SEG_KINDS:
            raise ValueError("no analytic Crofton weight for orbit segments of kind %r" % s["kind"])
        a, b = _SEG_PARAMS[s["kind"]]
        buf[i] = _lib.DcOrbitSegment(_SEG_KINDS[s["kind"]], int(s["start"]), int(s["count"]), int(bool(s["closed"])),
                                     float(s[a]), float(s[b]), float(s.get("phi_max", 0.0)), float(s.get("freq", 0.0)))
    return buf


def dc_crofton_weights(plan, segments, sid, M, m_exp=2, taper=0.05, c_floor=0.01, fine=64, v0=0, nv=None,
                       stream=None):
    """Smooth Crofton weight of eq. 9 into M [V][n_theta][n_s] for views [v0, v0+nv)."""
    _need(M, "M", (plan.n_views,) + plan.sino_shape)
    v0, nv = _range(plan, v0, nv)
    segs = make_segments(segments)
    L = _lib.lib()
    nbytes = L.dc_crofton_workspace_bytes(segs, len(segs), int(fine))
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=M.device)
    check(L.dc_crofton_weights(plan.handle, segs, len(segs), float(sid), int(m_exp), float(taper), float(c_floor),
                               int(fine), _ptr(M), v0, nv, _ptr(work), nbytes, _stream(stream)),
          "dc_crofton_weights")
    return M


def dc_poisson_noise(p, out, photons, mu, seed, counts=None, e0=0, stream=None):
    """Poisson-noisy line integrals of p (any float32 shape, contiguous) into out
    (may be p); counts (int64, same shape, optional) receives the photon counts."""
    if not p.is_contiguous() or p.dtype != torch.float32 or out.shape != p.shape or out.dtype != torch.float32:
        raise ValueError("p and out must be contiguous float32 arrays of one shape")
    if counts is not None and (counts.shape != p.shape or counts.dtype != torch.int64 or not counts.is_contiguous()):
        raise ValueError("counts must be a contiguous int64 array of p's shape")
    check(_lib.lib().dc_poisson_noise(_ptr(p), _ptr(out), _ptr(counts), p.numel(), float(photons), float(mu),
                                      int(seed) & (2**64 - 1), int(e0), _stream(stream)), "dc_poisson_noise")
    return out


def dc_adam_step(M, G, m, v, step, lr, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.0, stream=None):
    """One fused Adam (AdamW if weight_decay > 0) step of M in place; m, v are the
    moment arrays and step a one-element float32 device tensor holding t >= 1."""
    for name, t in (("M", M), ("G", G), ("m", m), ("v", v)):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.shape != M.shape:
            raise ValueError("%s must be a contiguous float32 array of M's shape" % name)
    if step.dtype != torch.float32 or step.numel() != 1:
        raise ValueError("step must be a one-element float32 tensor")
    check(_lib.lib().dc_adam_step(_ptr(M), _ptr(G), _ptr(m), _ptr(v), M.numel(), _ptr(step), float(lr),
                                  float(betas[0]), float(betas[1]), float(eps), float(weight_decay), _stream(stream)),
          "dc_adam_step")
    return M


def dc_ssim(x, y, data_range, grad=False, stream=None):
    """Mean 3D SSIM of x against y (volumes [nz][ny][nx]) and, with grad=True, its
    gradient w.r.t. x.  Returns (ssim as a 1-element tensor, grad or None)."""
    if x.dim() != 3 or tuple(x.shape) != tuple(y.shape):
        raise ValueError("x and y must be volumes of one shape")
    _need(x, "x", tuple(x.shape))
    _need(y, "y", tuple(y.shape))
    nz, ny, nx = x.shape
    L = _lib.lib()
    nbytes = L.dc_ssim_workspace_bytes(nz, ny, nx)
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=x.device)
    out = torch.empty(1, dtype=torch.float32, device=x.device)
    g = torch.empty_like(x) if grad else None
    check(L.dc_ssim(_ptr(x), _ptr(y), nz, ny, nx, float(data_range), _ptr(out), _ptr(g), _ptr(work), nbytes,
                    _stream(stream)), "dc_ssim")
    return out, g


def dc_project(plan, vol, g, v0=0, nv=None, stream=None):
    """Siddon projections of the voxel volume: g[v] for views [v0, v0+nv)."""
    _need(vol, "vol", plan.vol_shape)
    _need(g, "g", (plan.n_views,) + plan.det_shape)
    v0, nv = _range(plan, v0, nv)
    check(_lib.lib().dc_project(plan.handle, _ptr(vol), _ptr(g), v0, nv, _stream(stream)), "dc_project")
    return g
