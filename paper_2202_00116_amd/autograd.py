"""Differentiable forms of the DEAM forward model (hand-written adjoints).

DEAMNLL:      c -> L(c) = sum over rays off the metal trace of g_j - d_j ln g_j
              (the Poisson negative log-likelihood, equal to the I-divergence
              of Eq. 5 up to a constant).  Its gradient is b~_i - b^_i =
              H^T u_i with u_i = sum_j (r_j - 1) a_ij (a_ij = sum_E mu_i q_j),
              so the backward pass is one 2-channel backprojection.
PolyForward:  c -> g (2, R), the expected counts of Eq. 8.  Its vector-Jacobian
              product for an upstream v = dloss/dg is -H^T sum_j v_j a_ij
              (one poly-mean pass in VJP mode and one backprojection).

DEAMStep:     c -> Phi(c) = c - ln(b~(c)/b^(c))/Z, one DEAM iteration on the
              FP64 image (2, V).  Its vector-Jacobian product (deam_iterate_vjp)
              recomputes the projections of c (only c is kept per iteration)
              and costs three forward projections and two backprojections;
              unrolled_deam chains n iterations, so that a loss on the
              reconstruction (a learned prior, a task loss) can be
              differentiated through the reconstruction itself.

All keep every step on the GPU library; torch only carries the tensors.
"""
from __future__ import annotations

import torch

from . import _lib as L


class DEAMNLL(torch.autograd.Function):
    """loss = DEAMNLL.apply(c, plan, d, mask); c: (2, V) in the plan dtype."""

    @staticmethod
    def forward(ctx, c, plan, d, mask):
        l = plan.forward(c.detach().contiguous())
        u, _, obj = plan.poly_mean(l, d, mask, mode=L.W_GRAD, want_obj=True)
        ctx.plan = plan
        ctx.save_for_backward(u)
        return obj.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        (u,) = ctx.saved_tensors
        grad = ctx.plan.backproject(u)
        return grad * grad_out.to(grad.dtype), None, None, None


class PolyForward(torch.autograd.Function):
    """g = PolyForward.apply(c, plan): expected counts (2, R) of the model."""

    @staticmethod
    def forward(ctx, c, plan):
        l = plan.forward(c.detach().contiguous())
        dummy = torch.zeros((2, plan.R), dtype=torch.float32, device=c.device)
        _, g, _ = plan.poly_mean(l, dummy, None, mode=L.W_AM, want_g=True)
        ctx.plan = plan
        ctx.save_for_backward(l)
        return g

    @staticmethod
    def backward(ctx, grad_g):
        (l,) = ctx.saved_tensors
        plan = ctx.plan
        v = grad_g.to(plan.dtype).contiguous()
        u, _, _ = plan.poly_mean(l, None, None, mode=L.W_VJP, v=v)
        return plan.backproject(u), None


class DEAMStep(torch.autograd.Function):
    """c_next = DEAMStep.apply(c, plan, d, mask, Z); c: float64 (2, V)."""

    @staticmethod
    def forward(ctx, c, plan, d, mask, Z):
        c_next = c.detach().clone().contiguous()
        plan.iterate(c_next, d, mask, Z, 1)
        ctx.plan, ctx.d, ctx.mask, ctx.Z = plan, d, mask, Z
        ctx.save_for_backward(c.detach())
        return c_next

    @staticmethod
    def backward(ctx, grad):
        (c,) = ctx.saved_tensors
        G = grad.to(torch.float64).contiguous()
        return ctx.plan.iterate_vjp(c.contiguous(), ctx.d, ctx.mask, ctx.Z, G), None, None, None, None


def unrolled_deam(c0, plan, d, mask, Z, n_iter):
    """n_iter differentiable DEAM iterations from c0 (float64 (2, V))."""
    c = c0
    for _ in range(n_iter):
        c = DEAMStep.apply(c, plan, d, mask, Z)
    return c
