"""Training of the redundancy weight M as the paper sets it up (Sec. 3.1, eq. 13).

    W      = G_sigma * M                       (Gaussian filter layer, sigma 20, 121 taps)
    f      = ReLU(DC-FBP(g; W))                (eq. 12 with the learned weight)
    L      = MSE(f', r') + gamma (1 - SSIM(f', r'))   on f' = f / max(r), r' = r / max(r)
    M init U[-1, 0] (RAW mode: W is the whole redundancy weight of eq. 10),
    AdamW with a one-cycle learning rate between 0.1 and 1.

Every step of the reconstruction, its transpose, the smoothing layer, the SSIM
term and the AdamW update runs in the HIP library; this module only wires them
to torch's autograd and learning-rate schedule.
"""
from __future__ import annotations

import torch

from . import ops
from .autograd import reconstruct, sinogram


class _SSIM(torch.autograd.Function):
    """1 - SSIM(x, y) with d/dx from the library (y is data, no gradient)."""

    @staticmethod
    def forward(ctx, x, y, data_range):
        s, g = ops.dc_ssim(x.contiguous(), y.contiguous(), data_range, grad=x.requires_grad)
        ctx.save_for_backward(g)
        return 1.0 - s[0]

    @staticmethod
    def backward(ctx, go):
        (g,) = ctx.saved_tensors
        return -go * g, None, None


class FusedAdamW(torch.optim.Optimizer):
    """AdamW whose update is the library's fused one-pass step (``dc_adam_step``);
    the step count is kept on the device.  Parameter groups carry ``lr`` and
    ``betas`` like torch's optimisers, so learning-rate (and momentum) schedules
    apply unchanged.  Parameters must be contiguous float32 device tensors."""

    def __init__(self, params, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.0):
        super().__init__(params, dict(lr=lr, betas=betas, eps=eps, weight_decay=weight_decay))

    @torch.no_grad()
    def step(self, closure=None):
        loss = closure() if closure is not None else None
        for group in self.param_groups:
            for p in group["params"]:
                if p.grad is None:
                    continue
                st = self.state[p]
                if not st:
                    st["m"], st["v"] = torch.zeros_like(p), torch.zeros_like(p)
                    st["step"] = torch.zeros(1, device=p.device)
                st["step"].add_(1.0)
                ops.dc_adam_step(p, p.grad.contiguous(), st["m"], st["v"], st["step"], group["lr"],
                                 group["betas"], group["eps"], group["weight_decay"])
        return loss


def ssim_loss(x, y, data_range=1.0):
    """1 - SSIM of volume x against y ([nz][ny][nx], or [S][nz][ny][nx] averaged over samples)."""
    if x.dim() == 4:
        return sum(_SSIM.apply(x[s], y[s], data_range) for s in range(x.shape[0])) / x.shape[0]
    return _SSIM.apply(x, y, data_range)


def paper_loss(f, ref, gamma=0.5):
    """Eq. 13 after normalising both volumes by the reference's maximum."""
    scale = 1.0 / float(ref.max())
    fn, rn = f * scale, ref * scale
    return torch.mean((fn - rn) ** 2) + gamma * ssim_loss(fn, rn.detach(), 1.0)


def train_weights(plan, g, ref, steps, gamma=0.5, smooth=(20.0, 60), lr=(0.1, 1.0), weight_decay=0.0,
                  store_dtype=torch.float32, seed=0, M0=None, callback=None):
    """Learns M in RAW mode for ``steps`` AdamW steps under a one-cycle schedule that
    starts and ends at lr[0] and peaks at lr[1].  Returns (M, list of losses)."""
    V = plan.n_views
    if M0 is None:
        gen = torch.Generator(device=g.device).manual_seed(seed)
        M0 = -torch.rand((V,) + plan.sino_shape, device=g.device, generator=gen)   # U[-1, 0]
    M = M0.clone().requires_grad_(True)
    R = sinogram(plan, g)                     # depends on the data only
    opt = FusedAdamW([M], lr=lr[0], weight_decay=weight_decay)
    sched = torch.optim.lr_scheduler.OneCycleLR(opt, max_lr=lr[1], total_steps=max(2, steps),
                                                div_factor=lr[1] / lr[0], final_div_factor=1.0)
    losses = []
    for it in range(steps):
        opt.zero_grad(set_to_none=True)
        f = reconstruct(plan, M, R=R, mode="raw", store_dtype=store_dtype, relu=True, smooth=smooth)
        loss = paper_loss(f, ref, gamma)
        loss.backward()
        opt.step()
        sched.step()
        losses.append(float(loss.detach()))
        if callback:
            callback(it, losses[-1])
    return M.detach(), losses
