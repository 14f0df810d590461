"""Differentiable forward model: the simulation y = A(theta) X wrapped in a
torch.autograd.Function whose backward runs the library's adjoint kernels
(d/dX through the gather back-projection, d/dtheta through
pvr_simulate_grad_theta).  FP64 and FP32 tensors select the matching entry
points.
"""
from __future__ import annotations

import torch

from . import pvr


class SimulateFn(torch.autograd.Function):
    """y_sim = A(theta) X for every sample of the plan (0 for invalid ones).

    Inputs: X [V] and theta [M, 6] on the GPU, same dtype (float32 or
    float64), and the plan (not differentiated).  The plan is rebuilt at
    theta in forward and, if it was rebuilt elsewhere in between, again in
    backward."""

    @staticmethod
    def forward(ctx, X, theta, plan):
        th = theta.detach().contiguous()
        plan.build(th)
        y = torch.empty(plan.N, dtype=X.dtype, device=X.device)
        plan.simulate(X.detach().contiguous(), y_sim=y)
        ctx.plan = plan
        ctx.build_id = plan.build_id
        ctx.save_for_backward(X.detach(), th)
        return y

    @staticmethod
    def backward(ctx, gy):
        X, th = ctx.saved_tensors
        plan = ctx.plan
        if plan.build_id != ctx.build_id:
            plan.build(th)
            ctx.build_id = plan.build_id
        gy = gy.contiguous()
        gX = gth = None
        if ctx.needs_input_grad[0]:
            gX = torch.empty_like(X)
            plan.backproject(gy, None, None, gX, None)
        if ctx.needs_input_grad[1]:
            gth = torch.empty_like(th)
            plan.grad_theta(X.contiguous(), gy, gth)
        return gX, gth, None


def simulate(X, theta, plan):
    return SimulateFn.apply(X, theta, plan)
