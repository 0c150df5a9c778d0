"""Differentiable solve x = A^-1 b through the library (the adjoint of the
refinement, as a torch.autograd.Function).

Forward: gmresir_factor + gmresir_solve.  Backward, for an upstream gradient
g = dL/dx: the adjoint system A^T lambda = g is solved by
gmresir_solve_transposed with the same (transposed) factors and a recycle
space of its own; then dL/db = lambda and dL/dA = -lambda x^T (gmresir_rank1).
Every arithmetic step runs in the HIP library; this module only passes
pointers.
"""
from __future__ import annotations

import torch

from . import GmresirError, STATUS, factor, rank1

__all__ = ["GmresirSolve", "solve"]


class GmresirSolve(torch.autograd.Function):
    """x = A^-1 b with A (n x n, row-major float64 CUDA) and b (n,)."""

    @staticmethod
    def forward(ctx, a, b, opts):
        h = factor(a.detach(), **opts)
        if h.status != 0:
            status = h.status
            h.free()
            raise GmresirError(status, f"factorisation: {STATUS.get(status, status)}")
        x, info = h.solve(b.detach().contiguous())
        ctx.handle = h
        ctx.info = info
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        h = ctx.handle
        try:
            lam, info = h.solve_transposed(gx.contiguous())
        finally:
            h.free()
        ctx.adjoint_info = info
        ga = rank1(-1.0, lam, x) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return ga, gb, None


def solve(a, b, **opts):
    """Differentiable x = A^-1 b (one backward pass per forward: the factors
    are released after the adjoint solve).  Options as for ``factor``."""
    return GmresirSolve.apply(a, b, opts)
