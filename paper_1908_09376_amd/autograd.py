"""torch.autograd.Function around the MIDBF apply.

forward:  g = K f            (midbf_apply)
backward: grad_f = K^H grad_g (midbf_apply_adjoint)

PyTorch's complex gradients are conjugate-Wirtinger: for a real loss L and a
linear map g = K f, the gradient it propagates is grad_f = K^H grad_g
(e.g. L = ||K f - y||^2 gives grad_f = 2 K^H (K f - y)).
"""
from __future__ import annotations

import torch


class MIDBFMatvec(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f: torch.Tensor, factor, precision: str):
        ctx.factor = factor
        ctx.precision = precision
        return factor.apply(f.contiguous(), precision=precision)

    @staticmethod
    def backward(ctx, grad_g: torch.Tensor):
        grad_f = ctx.factor.apply_adjoint(grad_g.contiguous(), precision=ctx.precision)
        return grad_f, None, None


def midbf_matvec(f: torch.Tensor, factor, precision: str = "fp64") -> torch.Tensor:
    """Differentiable g = K f for f of shape (N,) or (nrhs, N)."""
    return MIDBFMatvec.apply(f, factor, precision)
