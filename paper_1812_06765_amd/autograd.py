"""Differentiation form: the objective J(y, T) = D(R, T(P y)) + alpha S(y) as a
torch.autograd.Function.

The forward and the hand-written backward both run in the HIP library
(``ngf_eval_pair``): the backward recomputes the warp and the NGF
sensitivity and scatters them with atomics into grad y (through P^T) and
grad T (through the transpose of the trilinear warp), scaled on the device
by the upstream gradient.  R is a constant of the objective.
"""

from __future__ import annotations

import torch


class NGFObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, T, R, h, lib_ctx):
        if R.requires_grad:
            raise ValueError("the reference image is a constant of the objective")
        J = torch.empty((), dtype=torch.float64, device=y.device)
        lib_ctx.eval_pair(R, T.detach(), y.detach(), h, grad_y=False, grad_T=False, J_dev=J,
                          sync=False)
        ctx.save_for_backward(y, T, R)
        ctx.h = h
        ctx.lib = lib_ctx
        return J

    @staticmethod
    def backward(ctx, gJ):
        y, T, R = ctx.saved_tensors
        scale = gJ.detach().reshape(1).contiguous()
        if scale.dtype != torch.float64:
            raise TypeError("the upstream gradient of J must be float64")
        _, gy, gT = ctx.lib.eval_pair(R, T.detach(), y.detach(), ctx.h,
                                      grad_y=ctx.needs_input_grad[0],
                                      grad_T=ctx.needs_input_grad[1], gscale=scale, sync=False)
        return gy, gT, None, None, None


def ngf_objective(y, T, R, h, lib_ctx):
    """J as a float64 0-d tensor, differentiable with respect to y and T."""
    return NGFObjective.apply(y, T, R, tuple(float(v) for v in h), lib_ctx)
