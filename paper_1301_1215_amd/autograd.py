"""F(rho, chat; P) as a torch.autograd.Function.

forward = nlinv_forward (Eq. 2).  backward = the hand-written adjoint:
F is complex-bilinear in (rho, chat) with no conjugation, so with torch's
convention for complex gradients (grad = dL/dRe + i dL/dIm) the vector-
Jacobian product is DF_x^H g (nlinv_adjoint); the gradient with respect to
the real sampling weights P is Re sum_j conj(g_j) . DTFT(E(rho . c_j))
(nlinv_mask_gradient).  Both run on the GPU kernels; nothing is traced.
"""
from __future__ import annotations

import torch

from .nlinv import Plan


class NlinvForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, chat, P, plan: Plan):
        rho, chat, P = rho.contiguous(), chat.contiguous(), P.contiguous()
        y, c = plan.forward(rho, chat, P, return_c=True)
        ctx.save_for_backward(rho, chat, P, c)
        ctx.plan = plan
        return y

    @staticmethod
    def backward(ctx, g):
        rho, chat, P, c = ctx.saved_tensors
        plan = ctx.plan
        g = g.contiguous()
        grho = gchat = gP = None
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            grho, gchat = plan.adjoint(rho, chat, P, g, c=c)
        if ctx.needs_input_grad[2]:
            gP = plan.mask_gradient(rho, chat, g, c=c)
        return grho, gchat, gP, None


def nlinv_F(rho, chat, P, plan: Plan):
    """Differentiable y = F(rho, chat; P) on the plan's frame shape."""
    return NlinvForward.apply(rho, chat, P, plan)
