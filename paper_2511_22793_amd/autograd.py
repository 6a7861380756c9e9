"""torch.autograd seam around the HIP renderer: forward and backward both run
in the library (gs_render_forward / gs_render_backward); this module only
keeps the workspace between them."""
from __future__ import annotations

from typing import Optional

import torch

from .render import Grid, Params, backward, forward


class GSRender(torch.autograd.Function):
    """spectrum = GSRender.apply(mean, log_scale, quat, opacity_logit, attr,
    rx, tx, grid, params, is_complex).  Differentiable in the four Gaussian
    parameter tensors and attr; rx / tx are constants."""

    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity_logit, attr, rx, tx: Optional[torch.Tensor], grid: Grid,
                params: Params, is_complex: bool):
        scene = {"mean": mean.detach().contiguous(), "log_scale": log_scale.detach().contiguous(),
                 "quat": quat.detach().contiguous(), "opacity_logit": opacity_logit.detach().contiguous()}
        a = attr.detach().contiguous()
        out, ws = forward(scene, a, rx, tx, grid=grid, params=params, is_complex=is_complex)
        ctx.ws, ctx.scene, ctx.attr, ctx.rx, ctx.tx, ctx.is_complex = ws, scene, a, rx, tx, is_complex
        ctx.out = out
        return out

    @staticmethod
    def backward(ctx, grad_out):
        g = backward(ctx.ws, ctx.scene, ctx.attr, ctx.rx, ctx.out, grad_out.contiguous(), tx=ctx.tx,
                     is_complex=ctx.is_complex)
        return (g["d_mean"], g["d_log_scale"], g["d_quat"], g["d_opacity_logit"], g["d_attr"], None, None, None,
                None, None)


def render(mean, log_scale, quat, opacity_logit, attr, rx, tx=None, grid: Grid = Grid(), params: Params = Params(),
           is_complex: bool = False):
    return GSRender.apply(mean, log_scale, quat, opacity_logit, attr, rx, tx, grid, params, is_complex)
