"""torch.autograd.Function around splat_trace / splat_trace_backward.

The forward saves only the output image; the backward re-traverses the BVH
to recompute each pixel's ordered hit list (nothing per hit is stored).
Gradients are per sphere: straight RGB, alpha a, radius and centre (the last
two are zero in constant-alpha mode, where the image is piecewise constant
in them).
"""
from __future__ import annotations

import torch

from . import _lib
from .render import BVH, Spheres, TraceOptions, trace, trace_backward


class SplatTrace(torch.autograd.Function):
    """out = trace(centre_radius, rgba); the BVH must match the current centres and radii.

    centre_radius float32 [N, 4] (x, y, z, r) and rgba float32 [N, 4]
    (straight r, g, b, a), both CUDA; `bvh` was built (or refit) over them.
    """

    @staticmethod
    def forward(ctx, centre_radius: torch.Tensor, rgba: torch.Tensor, bvh: BVH, cam, opts: TraceOptions,
                count: torch.Tensor):
        sph = Spheres(centre_radius.detach(), rgba.detach(), count)
        out, _ = trace(bvh, sph, cam, opts, want_hits=False)
        ctx.save_for_backward(centre_radius.detach(), rgba.detach(), count, out)
        ctx.bvh, ctx.cam, ctx.opts = bvh, cam, opts
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        cr, rgba, count, out = ctx.saved_tensors
        sph = Spheres(cr, rgba, count)
        g = trace_backward(ctx.bvh, sph, ctx.cam, ctx.opts, out, grad_out.contiguous().float())
        d_cr = torch.cat([g["centre"], g["radius"][:, None]], dim=1)
        d_rgba = torch.cat([g["rgb"], g["alpha"][:, None]], dim=1)
        if ctx.opts.mode != _lib.SPLAT_ALPHA_SOFT:
            d_cr = torch.zeros_like(d_cr)
        return d_cr, d_rgba, None, None, None, None


def splat_trace(centre_radius: torch.Tensor, rgba: torch.Tensor, bvh: BVH, cam, opts: TraceOptions | None = None,
                count: torch.Tensor | None = None) -> torch.Tensor:
    """Differentiable trace; returns the [H, W, 4] premultiplied image."""
    opts = opts or TraceOptions(mode=_lib.SPLAT_ALPHA_SOFT)
    if count is None:
        count = torch.full((1,), centre_radius.shape[0], dtype=torch.int32, device=centre_radius.device)
    return SplatTrace.apply(centre_radius, rgba, bvh, cam, opts, count)
