"""torch.autograd.Function wrapper: forward = ppt_render, backward = ppt_backward."""
from __future__ import annotations

import torch


class PolarizedRender(torch.autograd.Function):
    """stokes = PolarizedRender.apply(plan, seed, backward_seed, *params)

    ``backward_seed`` None replays the rendered paths exactly (the derivative of this very
    estimate); another value gives the decorrelated replay of path replay backpropagation
    (phase 2 uses new paths), which is unbiased for non-linear losses.
    """

    @staticmethod
    def forward(ctx, plan, seed, backward_seed, *params):
        out = plan.render(list(params), seed)
        ctx.plan = plan
        ctx.seed = seed if backward_seed is None else backward_seed
        ctx.save_for_backward(*params)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        params = ctx.saved_tensors
        want = list(ctx.needs_input_grad[3:])
        grads = ctx.plan.backward(list(params), ctx.seed, grad_out.contiguous(), want=want)
        return (None, None, None, *grads)


def render(plan, params, seed, backward_seed=None):
    return PolarizedRender.apply(plan, seed, backward_seed, *params)
