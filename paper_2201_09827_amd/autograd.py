"""Differentiable solve x = A^-1 b through the library (the adjoint of the
refinement, as a torch.autograd.Function).

Forward: gmresir_factor + gmresir_solve.  Backward, for an upstream gradient
g = dL/dx: the adjoint system A^T lambda = g is solved by
gmresir_solve_transposed with the same (transposed) factors and a recycle
space of its own; then dL/db = lambda and dL/dA = -lambda x^T (gmresir_rank1).
Every arithmetic step runs in the HIP library; this module only passes
pointers.

A solve that does not reach the backward-error target (ENOCONV), or any other
nonzero status, raises GmresirError in forward or in backward: its x (or
lambda) would otherwise flow on as if it were the solution.  The error
carries the solve's record as ``.info``; with ``records=`` the caller also
gets the records of successful solves (keys "forward" and "adjoint").
"""
from __future__ import annotations

import torch

from . import GmresirError, STATUS, factor, rank1

__all__ = ["GmresirSolve", "solve"]


def _check(info: dict, what: str):
    st = int(info["status"])
    if st != 0:
        err = GmresirError(st, f"{what}: {STATUS.get(st, st)} after {info['steps']} refinement "
                               f"steps (Arnoldi steps {info['its']}, backward error "
                               f"{info['berr'][-1]:.3e})")
        err.info = info
        raise err


class GmresirSolve(torch.autograd.Function):
    """x = A^-1 b with A (n x n, row-major float64 CUDA) and b (n,)."""

    @staticmethod
    def forward(ctx, a, b, opts, records):
        h = factor(a.detach(), **opts)
        if h.status != 0:
            status = h.status
            h.free()
            raise GmresirError(status, f"factorisation: {STATUS.get(status, status)}")
        try:
            x, info = h.solve(b.detach().contiguous())
            if records is not None:
                records["forward"] = info
            _check(info, "forward solve")
        except BaseException:
            h.free()
            raise
        ctx.handle = h
        ctx.records = records
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
        if ctx.records is not None:
            ctx.records["adjoint"] = info
        _check(info, "adjoint solve")
        ga = rank1(-1.0, lam, x) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return ga, gb, None, None


def solve(a, b, records: dict | None = None, **opts):
    """Differentiable x = A^-1 b (one backward pass per forward: the factors
    are released after the adjoint solve).  Options as for ``factor``.
    ``records``, if given, receives the info dicts of the forward and the
    adjoint solve.  Raises GmresirError when either solve ends with a nonzero
    status (ENOCONV included)."""
    return GmresirSolve.apply(a, b, opts, records)
