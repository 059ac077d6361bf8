"""Differentiable forward model: torch.autograd over pat_forward.

g = A f with gradients with respect to the image f (pat_adjoint applied to
dL/dg) and to the sensor positions (sum over samples of dL/dg times the
traces' position derivatives from pat_forward_dxy). Positions enter the
plan's tables, so a plan serves one geometry: the gradient with respect to
the positions is the derivative at the positions the plan was built for.
"""
from __future__ import annotations

import numpy as np
import torch


class _Forward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, sensor_xy, plan):
        ctx.plan = plan
        ctx.xy_meta = (sensor_xy.device, sensor_xy.dtype)
        ctx.save_for_backward(f)
        return plan.forward(f.contiguous())

    @staticmethod
    def backward(ctx, grad_g):
        (f,) = ctx.saved_tensors
        plan = ctx.plan
        grad_g = grad_g.contiguous()
        gf = gxy = None
        if ctx.needs_input_grad[0]:
            gf = plan.adjoint(grad_g)
        if ctx.needs_input_grad[1]:
            fc = f.contiguous()
            dx = plan.forward_dxy(fc, 0)
            dy = plan.forward_dxy(fc, 1)
            gxy = torch.stack(((grad_g * dx).sum(dim=1), (grad_g * dy).sum(dim=1)), dim=1)
            gxy = gxy.to(device=ctx.xy_meta[0], dtype=ctx.xy_meta[1])
        return gf, gxy, None


def forward_model(f, sensor_xy, plan):
    """g = A f (pat_forward), differentiable in f and in sensor_xy.

    f: [Nx, Ny, Nz] tensor on the plan's device in its precision.
    sensor_xy: [M, 2] tensor holding the positions the plan was built for
    (any device; checked against the plan's copy).
    """
    xy = sensor_xy.detach().to("cpu", torch.float64).numpy()
    if xy.shape != plan.sensor_xy.shape or not np.array_equal(xy, plan.sensor_xy):
        raise ValueError("sensor_xy differs from the positions the plan was built for")
    return _Forward.apply(f, sensor_xy, plan)
