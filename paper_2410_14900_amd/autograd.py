"""Differentiable reconstruction f(M) of eq. 12 with exact gradients w.r.t. M.

Forward: R = A2d(w_cos g) (cached or recomputed), H = D(W D R), gF = A2d^T H,
f = cone-beam BP of gF (+ ReLU).  Backward (f is linear in M): the HIP adjoint
kernels apply the transposes in reverse order and dc_filter_adjoint forms dL/dM.
"""
from __future__ import annotations

import torch

from . import ops


def sinogram(plan, g, dtype=torch.float32, out=None):
    """R = A2d(w_cos g) for all views (depends on the data only, not on M)."""
    V = plan.n_views
    R = out if out is not None else torch.empty((V,) + plan.sino_shape, device=g.device, dtype=dtype)
    return ops.dc_weight_radon(plan, g, R)


class _DCFBP(torch.autograd.Function):
    @staticmethod
    def forward(ctx, M, R, g, plan, mode, store_dtype, relu, recompute_R, smooth):
        V = plan.n_views
        dev = M.device
        if R is None:
            R = sinogram(plan, g)
        Mw = M
        if smooth is not None:
            Mw = ops.dc_smooth_weights(plan, M, torch.empty_like(M), *smooth)
        H = torch.empty((V,) + plan.sino_shape, device=dev, dtype=store_dtype)
        ops.dc_filter(plan, R, Mw, H, mode=mode)
        gF = torch.empty((V,) + plan.det_shape, device=dev, dtype=store_dtype)
        ops.dc_detector_bp(plan, H, gF)
        del H
        f = torch.empty(plan.vol_shape, device=dev, dtype=torch.float32)
        ops.dc_cone_bp(plan, gF, f, relu=relu)
        ctx.plan, ctx.mode, ctx.store_dtype, ctx.relu, ctx.recompute_R = plan, mode, store_dtype, relu, recompute_R
        ctx.smooth = smooth
        saved_R = None if recompute_R else R
        ctx.save_for_backward(Mw, saved_R, g if recompute_R else None, f if relu else None)
        return f

    @staticmethod
    def backward(ctx, Gf):
        M, R, g, f = ctx.saved_tensors
        plan = ctx.plan
        V = plan.n_views
        dev = M.device
        if R is None:
            R = sinogram(plan, g)
        GgF = torch.empty((V,) + plan.det_shape, device=dev, dtype=ctx.store_dtype)
        ops.dc_cone_bp_adjoint(plan, Gf.contiguous(), GgF, f_relu=f)
        GH = torch.empty((V,) + plan.sino_shape, device=dev, dtype=ctx.store_dtype)
        ops.dc_detector_bp_adjoint(plan, GgF, GH)
        del GgF
        GM = torch.empty_like(M)
        ops.dc_filter_adjoint(plan, GH, R, M, GM=GM, mode=ctx.mode)
        if ctx.smooth is not None:
            ops.dc_smooth_weights_adjoint(plan, GM, GM, *ctx.smooth)
        return GM, None, None, None, None, None, None, None, None


def reconstruct(plan, M, g=None, R=None, mode="analytic", store_dtype=torch.float32, relu=False,
                recompute_R=False, smooth=None):
    """f = DC-FBP(g; M).  Pass the sinogram R (from ``sinogram``) to reuse it
    across steps, or g to compute it; recompute_R keeps only g for the backward.
    smooth = (sigma, radius) inserts the Gaussian filter layer on M (Sec. 3.1:
    (20.0, 60)) before the weight is used; its transpose runs in the backward."""
    if R is None and g is None:
        raise ValueError("need g or R")
    if recompute_R and g is None:
        raise ValueError("recompute_R needs g")
    return _DCFBP.apply(M, R, g, plan, mode, store_dtype, relu, recompute_R,
                        None if smooth is None else (float(smooth[0]), int(smooth[1])))


class DCFBP:
    """The DC-FBP layer with its settings fixed: ``DCFBP(plan, mode, dtype,
    recompute_R).apply(g, M)`` is ``reconstruct(plan, M, g=g, ...)`` (f, with exact
    gradients for M through the chain of transposes)."""

    def __init__(self, plan, mode="analytic", dtype=torch.float32, recompute_R=False, relu=False, smooth=None):
        self.plan, self.mode, self.dtype = plan, mode, dtype
        self.recompute_R, self.relu, self.smooth = recompute_R, relu, smooth

    def apply(self, g, M):
        return reconstruct(self.plan, M, g=g, mode=self.mode, store_dtype=self.dtype, relu=self.relu,
                           recompute_R=self.recompute_R, smooth=self.smooth)
