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

from . import _native as N
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


class GaussNewtonStep(torch.autograd.Function):
    """x_{n+1} = x_n + dx, (DF^H DF + alpha I) dx = DF^H (y - F x_n) - alpha (x_n - x_ref)
    (Eq. 3), differentiable with respect to the data y, the sampling weights P,
    the regularisation weight alpha, the references x_ref and the
    linearisation point x_n (implicit differentiation: the backward solves the
    same normal equations for the incoming gradient on the GPU,
    nlinv_gn_step_vjp).  Forward and backward run cg_iters CG iterations."""

    @staticmethod
    def forward(ctx, y, P, alpha, rho_ref, chat_ref, rho_n, chat_n, plan: Plan, cg_iters: int):
        a = float(alpha)
        prm = plan.params(1, cg_iters, alpha0=a, alpha_q=1.0, scale_norm=0.0, warm_start=True)
        y, P, rho_ref, chat_ref = y.contiguous(), P.contiguous(), rho_ref.contiguous(), chat_ref.contiguous()
        rho_n, chat_n = rho_n.contiguous(), chat_n.contiguous()
        out = plan.solve(y, P, prm, rho0=rho_n, chat0=chat_n, rho_ref=rho_ref, chat_ref=chat_ref)
        ctx.save_for_backward(y, P, rho_ref, chat_ref, rho_n, chat_n, out["rho"], out["chat"])
        ctx.plan, ctx.alpha, ctx.cg_iters = plan, a, cg_iters
        ctx.alpha_dtype = alpha.dtype if torch.is_tensor(alpha) else torch.float32
        return out["rho"], out["chat"]

    @staticmethod
    def backward(ctx, g_rho, g_chat):
        y, P, rho_ref, chat_ref, rho_n, chat_n, rho1, chat1 = ctx.saved_tensors
        if g_rho is None:
            g_rho = torch.zeros_like(rho1)
        if g_chat is None:
            g_chat = torch.zeros_like(chat1)
        need = ctx.needs_input_grad
        gr = N.nlinv_gn_step_vjp(ctx.plan.handle, rho_n, chat_n, y, P, ctx.alpha, rho1, chat1, rho_ref, chat_ref,
                                 g_rho.contiguous(), g_chat.contiguous(), ctx.cg_iters, want_y=need[0],
                                 want_ref=need[3] or need[4], want_P=need[1], want_alpha=need[2],
                                 want_x_n=need[5] or need[6])
        ga = gr.get("alpha")
        return (gr.get("y"), gr.get("P"), None if ga is None else ga.to(ctx.alpha_dtype),
                gr.get("rho_ref"), gr.get("chat_ref"), gr.get("rho_n"), gr.get("chat_n"), None, None)


def gauss_newton_step(y, P, alpha, rho_ref, chat_ref, rho_n, chat_n, plan: Plan, cg_iters: int = 30):
    """Differentiable regularised Gauss-Newton step (Eq. 3) from x_n = (rho_n,
    chat_n); alpha a float or a 0-dim real tensor.  Returns (rho_{n+1}, chat_{n+1})."""
    return GaussNewtonStep.apply(y, P, alpha, rho_ref, chat_ref, rho_n, chat_n, plan, cg_iters)


def irgnm_unrolled(y, P, rho0, chat0, plan: Plan, newton_steps: int = 7, cg_iters: int = 30, alpha0=1.0,
                   alpha_q: float = 0.5, alpha_min: float = 0.0, rho_ref=None, chat_ref=None):
    """The Newton loop of Eq. 3 as a chain of differentiable steps:
    x_{k+1} = step(x_k; y, P, alpha_k, x_ref) with alpha_k = max(alpha0 q^k,
    alpha_min) and x_ref = x0 unless given, all in the units of y (no data
    scaling).  Gradients reach y, P, x0, x_ref and alpha0 (a float or a 0-dim
    real tensor) through every step; autograd keeps the iterates.  Returns
    (rho_N, chat_N)."""
    if rho_ref is None:
        rho_ref, chat_ref = rho0, chat0
    rho, chat = rho0, chat0
    for k in range(newton_steps):
        if torch.is_tensor(alpha0):
            a = torch.clamp_min(alpha0 * alpha_q ** k, alpha_min)
        else:
            a = max(alpha0 * alpha_q ** k, alpha_min)
        rho, chat = GaussNewtonStep.apply(y, P, a, rho_ref, chat_ref, rho, chat, plan, cg_iters)
    return rho, chat


def nlinv_F(rho, chat, P, plan: Plan):
    """Differentiable y = F(rho, chat; P) on the plan's frame shape."""
    return NlinvForward.apply(rho, chat, P, plan)
