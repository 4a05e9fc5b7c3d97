"""Fitting splat radii and opacities to a reference view through the
differentiable trace (soft alpha profile).

Parameters are log r and logit a per sphere; centres and colours stay fixed,
so every step only refits the BVH boxes (the hierarchy over the centres does
not change).  Adam runs in torch; trace, backward and refit run in the HIP
kernels.
"""
from __future__ import annotations

import torch

from . import _lib
from .autograd import splat_trace
from .render import BVH, Spheres, TraceOptions, build_bvh


def fit_radius_alpha(sph: Spheres, bvh: BVH, cam, reference: torch.Tensor, steps: int = 200, lr: float = 1e-2,
                     betas=(0.9, 0.999), alpha_stop: float = 0.99) -> list[float]:
    """Adam on (log r, logit a); returns the loss before every step and after the last one.

    `sph` must hold float32 colours; it is updated in place with the fitted
    radii and alphas, and `bvh` is refit to them.
    """
    if sph.half:
        raise ValueError("fit_radius_alpha needs float32 sphere colours")
    n = sph.n()
    cr = sph.centre_radius[:n]
    rgba = sph.rgba[:n]
    eps = 1e-6
    log_r = torch.log(cr[:, 3].clone()).requires_grad_(True)
    a0 = rgba[:, 3].clamp(eps, 1 - eps)
    logit_a = torch.log(a0 / (1 - a0)).requires_grad_(True)
    opt = torch.optim.Adam([log_r, logit_a], lr=lr, betas=betas)
    opts = TraceOptions(alpha_stop=alpha_stop, mode=_lib.SPLAT_ALPHA_SOFT)
    count = torch.full((1,), n, dtype=torch.int32, device=cr.device)
    losses = []
    for it in range(steps + 1):
        with torch.no_grad():
            cr[:, 3] = torch.exp(log_r)
            rgba[:, 3] = torch.sigmoid(logit_a)
        build_bvh(sph, bvh, refit_only=True)
        cr_in = torch.cat([cr[:, :3], torch.exp(log_r)[:, None]], dim=1)
        rgba_in = torch.cat([rgba[:, :3], torch.sigmoid(logit_a)[:, None]], dim=1)
        img = splat_trace(cr_in, rgba_in, bvh, cam, opts, count)
        loss = ((img - reference) ** 2).sum()
        losses.append(float(loss.detach()))
        if it == steps:
            break
        opt.zero_grad()
        loss.backward()
        opt.step()
    return losses
