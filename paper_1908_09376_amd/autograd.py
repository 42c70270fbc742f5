"""torch.autograd.Function around the MIDBF apply.

forward:  g = K f            (midbf_apply)
backward: grad_f = K^H grad_g (midbf_apply_adjoint, or midbf_apply of a factorization of K^H)

PyTorch's complex gradients are conjugate-Wirtinger: for a real loss L and a
linear map g = K f, the gradient it propagates is grad_f = K^H grad_g
(e.g. L = ||K f - y||^2 gives grad_f = 2 K^H (K f - y)).

The backward takes the forward factors' adjoint walk (FP64 or FP32; exactly
the adjoint of the forward approximation) unless a factorization of K^H is
given (built with adjoint=True): that one runs in any kept precision, the
split 16-bit ones included, and is the adjoint of K to the build tolerance.
"""
from __future__ import annotations

import torch


class MIDBFMatvec(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f: torch.Tensor, factor, precision: str, adjoint_factor, adjoint_precision: str):
        ctx.factor = factor
        ctx.precision = precision
        ctx.adjoint_factor = adjoint_factor
        ctx.adjoint_precision = adjoint_precision
        return factor.apply(f.contiguous(), precision=precision)

    @staticmethod
    def backward(ctx, grad_g: torch.Tensor):
        if ctx.adjoint_factor is not None:
            grad_f = ctx.adjoint_factor.apply(grad_g.contiguous(), precision=ctx.adjoint_precision)
        else:
            grad_f = ctx.factor.apply_adjoint(grad_g.contiguous(), precision=ctx.adjoint_precision)
        return grad_f, None, None, None, None


def midbf_matvec(f: torch.Tensor, factor, precision: str = "fp64", adjoint_factor=None,
                 adjoint_precision: str | None = None) -> torch.Tensor:
    """Differentiable g = K f for f of shape (N,) or (nrhs, N).  adjoint_factor: a factorization of
    K^H (adjoint=True, same points) for the backward; adjoint_precision: the backward's precision
    (default: the forward's)."""
    if adjoint_factor is not None and (adjoint_factor.N != factor.N or not adjoint_factor.adjoint
                                       or factor.adjoint):
        raise ValueError("adjoint_factor must be a factorization of K^H (adjoint=True) of the same size")
    return MIDBFMatvec.apply(f, factor, precision, adjoint_factor, adjoint_precision or precision)
