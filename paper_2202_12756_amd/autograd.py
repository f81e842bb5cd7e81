"""Differentiable forms of the transforms (hand-written adjoints).

With real inner products <F,G> = sum_{k in half} Re(conj F G) and
<f,h> = sum_j f h, and torch's gradient convention for complex tensors
(dL/dRe + i dL/dIm), the backward passes are the adjoints:
  * forward R2C  F = R2C(u)          : du = R2C^T(gF) = C2R(gF / w)
  * inverse C2R  f = s C2R(G)        : dG = s C2R^T(gf) = s w R2C(gf)
w(kz) = 1 at kz = 0 and kz = N/2, 2 otherwise: the stored half spectrum
counts every other bin twice (section 2, Hermitian symmetry of the
transform of a real field).  Both adjoints run in libgfft.so, with the
weights folded into the z passes.
"""
from __future__ import annotations

import torch

from .fft import Plan


class RFFT3(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u: torch.Tensor, plan: Plan):
        ctx.plan = plan
        return plan.r2c(u.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        plan = ctx.plan
        g = g.contiguous().clone()        # the adjoint clobbers its input
        return plan.r2c_adjoint(g, scale=1.0), None


class IRFFT3(torch.autograd.Function):
    @staticmethod
    def forward(ctx, G: torch.Tensor, plan: Plan, scale: float):
        ctx.plan = plan
        ctx.scale = scale
        return plan.c2r(G.contiguous().clone(), scale=scale)

    @staticmethod
    def backward(ctx, h: torch.Tensor):
        return ctx.plan.c2r_adjoint(h.contiguous(), scale=ctx.scale), None, None


def rfft3(u: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable forward R2C of a [batch, X, N, N] real tensor."""
    return RFFT3.apply(u, plan)


def irfft3(G: torch.Tensor, plan: Plan, scale: float = 1.0) -> torch.Tensor:
    """Differentiable inverse C2R (times ``scale``); ``G`` is not modified."""
    return IRFFT3.apply(G, plan, scale)
