"""Iterative reconstruction with the GPU forward model and its adjoint.

Landweber iteration f_{k+1} = f_k + tau A*(g - A f_k) from f_0 = 0, with
tau = 1/||A||^2 estimated by power iteration on A*A. A and A* are the
library's pat_forward / pat_adjoint; the vector updates are elementwise
device operations on the plan's stream.
"""
from __future__ import annotations

import torch


def operator_norm_sq(plan, x0, iters=20):
    """Largest eigenvalue of A*A by power iteration from the image x0:
    x <- A*A x / ||A*A x||; returns the Rayleigh quotient of the last iterate."""
    x = x0 / torch.linalg.vector_norm(x0)
    lam = 0.0
    for _ in range(iters):
        y = plan.adjoint(plan.forward(x))
        lam = float(torch.dot(x.reshape(-1), y.reshape(-1)))
        x = y / torch.linalg.vector_norm(y)
    return lam


def landweber(plan, g, iters=10, tau=None, x0=None, power_iters=20):
    """Landweber iterates for traces g. Returns (f, residual norms ||g - A f_k||
    for k = 0..iters, tau). With tau None it is 1/||A||^2 from power iteration
    started at x0 (required then: a seeded image of the plan's shape)."""
    if tau is None:
        if x0 is None:
            raise ValueError("x0 is needed to estimate ||A||^2")
        tau = 1.0 / operator_norm_sq(plan, x0, power_iters)
    f = torch.zeros(plan.shape, dtype=plan.dtype, device=plan.device)
    res = []
    for _ in range(iters):
        r = g - plan.forward(f)
        res.append(float(torch.linalg.vector_norm(r)))
        f = f + tau * plan.adjoint(r.contiguous())
    res.append(float(torch.linalg.vector_norm(g - plan.forward(f))))
    return f, res, tau
