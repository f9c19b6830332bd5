"""Differentiation layer: the forward map, its Born derivative and its adjoint
as a ``torch.autograd.Function``.

``forward(m) = f(m)`` (data of every shot, Section 2), ``backward`` applies
``F*`` (migration, eq. grad of Section 2.1) and ``jvp`` applies the Born
operator ``F``.  The forward pass keeps forward checkpoints every K steps in a
workspace held by the autograd context, so the backward pass recomputes the
forward wavefield segment by segment from them instead of solving the forward
again; the backward may be repeated (``retain_graph=True``).

All arithmetic runs in the HIP kernels behind the C ABI; this module only
routes tensors.  Gauss-Newton products are available as ``J^T (J v)`` through
autograd (vjp of jvp) and, fused and batched, as :func:`gn_hvp`.
"""
from __future__ import annotations

import torch

from . import fwi


class FwiForward(torch.autograd.Function):
    """d = f(m) for a :class:`fwi.Plan`; differentiable in m (reverse mode
    through the adjoint, forward mode through the Born operator)."""

    @staticmethod
    def forward(ctx, m, plan):
        ws = plan.new_workspace(fwi.FWI_OP_ADJOINT, 1)
        d = plan.forward_keep(m.detach(), ws)
        ctx.plan = plan
        ctx.ws = ws
        ctx.save_for_backward(m)
        ctx.save_for_forward(m)
        return d

    @staticmethod
    def backward(ctx, grad_d):
        plan = ctx.plan
        g = plan.adjoint_resume(grad_d.detach().float().contiguous(), ctx.ws)
        return g, None

    @staticmethod
    def jvp(ctx, m_dot, _plan_dot):
        (m,) = ctx.saved_tensors
        return ctx.plan.born(m.detach(), m_dot.detach().float().contiguous())


def forward(m, plan):
    return FwiForward.apply(m, plan)


def born_jvp(m, v, plan):
    """J v through forward-mode autograd (dual numbers)."""
    import torch.autograd.forward_ad as fwAD

    with fwAD.dual_level():
        out = FwiForward.apply(fwAD.make_dual(m.detach(), v.detach()), plan)
        return fwAD.unpack_dual(out).tangent


class Misfit(torch.autograd.Function):
    """Phi(m) = 1/2 inv_noise_var |f(m) - dobs|^2 (FP64 scalar).  One call to
    the fused misfit-gradient entry point computes Phi and its gradient; the
    gradient is kept for the backward pass."""

    @staticmethod
    def forward(ctx, m, dobs, plan):
        phi, grad = plan.misfit_grad(m.detach(), dobs.detach())
        ctx.save_for_backward(grad)
        return phi

    @staticmethod
    def backward(ctx, gphi):
        (grad,) = ctx.saved_tensors
        return (gphi.to(grad.dtype) * grad), None, None


def misfit(m, dobs, plan):
    return Misfit.apply(m, dobs, plan)


def gn_hvp_autograd(m, v, plan):
    """J^T Gamma^-1 J v through autograd: forward mode (Born) for J v, then
    reverse mode (adjoint) for J^T.  Same result as :func:`gn_hvp` up to
    rounding."""
    jv = born_jvp(m, v, plan)
    x = m.detach().requires_grad_(True)
    d = FwiForward.apply(x, plan)
    (hv,) = torch.autograd.grad(d, x, grad_outputs=jv)
    return hv * plan.geom.inv_noise_var


def gn_hvp(m, v, plan):
    """Fused, batched Gauss-Newton products H v for v[B][nz][nx]: one forward
    solve and its recompute shared by the batch."""
    return plan.gn_hvp(m.detach(), v.detach())
