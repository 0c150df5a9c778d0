"""LU factorisation with partial pivoting in precision u_f (oracle).

Test infrastructure only.  Follows the factorisation step of Algorithms 1-3
of the paper (an LU factorisation of A in precision u_f) with Gaussian
elimination with partial pivoting (GEPP, Section 1), written out step by step.

Build mode (:func:`lu_blocked`) fixes where rounding happens, which the paper
leaves open beyond naming the precision u_f:

* the matrix lives in u_f between block steps;
* a panel of ``nb`` columns is copied into the LU work precision wp (fp32 for
  fp16/bf16/fp32 storage, fp64 for fp64 storage) and eliminated column by
  column: the pivot is the first row index attaining max |a| in the current
  column; whole panel rows are swapped; the multipliers are
  fl_wp(a / pivot); every remaining panel entry is updated with one fused
  multiply-add fl_wp(a - l * u) per elimination step, in column order;
* the panel is written back rounded to u_f, the same row swaps are applied to
  the columns left and right of the panel;
* the block row to the right of the panel is solved with the stored (u_f)
  unit lower triangle, again one fused multiply-add per term in row order,
  and rounded to u_f;
* the trailing matrix receives A22 - L21 U12 computed from the stored u_f
  factors with (at least) fp32 accumulation, rounded once to u_f.  Here the
  product is formed in float64, which is exact or nearly so for u_f inputs;
  a GPU that accumulates in fp32 may differ by one u_f ulp on a small
  fraction of entries, so this step is compared by error bounds.

Paper mode (:func:`lu_chop`) is unblocked GEPP with every scalar product and
difference rounded to u_f, as a chop-style simulation does.

Pivots are returned LAPACK style: ``ipiv[i]`` is the row swapped with row i
at step i (0-based).  The permutation vector ``perm`` satisfies
(P b)[i] = b[perm[i]], so P A = L U.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .fp import fl, two_sum

__all__ = [
    "LUResult",
    "fp16_scale_exponent",
    "lu_blocked",
    "lu_chop",
    "perm_from_ipiv",
    "unpack",
    "fma_round",
]


@dataclass
class LUResult:
    lu: np.ndarray        # packed factors (float64 holding u_f values)
    ipiv: np.ndarray      # int64, LAPACK-style sequential swaps (0-based)
    info: int             # 0, or 1-based column of the first exact zero pivot
    uf: str

    @property
    def perm(self) -> np.ndarray:
        return perm_from_ipiv(self.ipiv)


def perm_from_ipiv(ipiv: np.ndarray) -> np.ndarray:
    n = ipiv.size
    p = np.arange(n)
    for i in range(n):
        j = int(ipiv[i])
        if j != i:
            p[i], p[j] = p[j], p[i]
    return p


def unpack(lu: np.ndarray):
    """Split packed factors into unit lower L and upper U (float64)."""
    n = lu.shape[0]
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    return L, U


def fp16_scale_exponent(amax: float, n: int = 1) -> int:
    """Largest integer e with 2^e * amax * sqrt(n) <= 2^-4 * 65504 (= 4094).

    Power-of-two scaling before rounding A to fp16 keeps the entries in the
    normal range at large n while leaving room for the element growth of
    partial pivoting (which grows roughly like sqrt(n) on dense random
    matrices); the scaling is exact and is undone in the preconditioner
    (M^-1 = 2^e U^-1 L^-1 P).
    """
    if not (amax > 0.0) or not math.isfinite(amax):
        return 0
    t = amax * math.sqrt(float(max(n, 1)))
    limit = 4094.0
    e = math.floor(math.log2(limit) - math.log2(t))
    while math.ldexp(t, e) > limit:
        e -= 1
    while math.ldexp(t, e + 1) <= limit:
        e += 1
    return int(e)


def _work_precision(uf: str) -> str:
    return "fp64" if uf == "fp64" else "fp32"


def _odd_round(s: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Round-to-odd of the exact value s + e (s = fl64(s + e))."""
    bits = s.view(np.int64)
    even = (bits & 1) == 0
    fix = (e != 0) & even & np.isfinite(s)
    out = s.copy()
    if np.any(fix):
        out[fix] = np.nextafter(s[fix], np.where(e[fix] > 0, np.inf, -np.inf))
    return out


def fma_round(a, b, c, prec: str) -> np.ndarray:
    """Correctly rounded fl_prec(a * b + c) for fp32 (or narrower) operands
    whose product is exact in float64 (<= 53 significant bits).

    The exact sum is rounded to odd at 53 bits, which makes the following
    rounding to a format with at most 51 bits correct (Boldo and Melquiond).
    For fp64 the plain float64 expression is returned.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    p = a * b
    if prec == "fp64":
        return p + c
    s, e = two_sum(c, p)
    s = np.asarray(s, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    return fl(_odd_round(np.atleast_1d(s), np.atleast_1d(e)).reshape(s.shape), prec)


def lu_blocked(af: np.ndarray, uf: str, nb: int) -> LUResult:
    """Blocked right-looking GEPP of ``af`` (float64 array of u_f values)."""
    a = np.array(af, dtype=np.float64, copy=True)
    n = a.shape[0]
    wp = _work_precision(uf)
    ipiv = np.arange(n, dtype=np.int64)
    info = 0
    for k0 in range(0, n, nb):
        kb = min(nb, n - k0)
        x = a[k0:, k0:k0 + kb].copy()            # exact in wp
        h = x.shape[0]
        for j in range(kb):
            col = np.abs(x[j:, j])
            p = j + int(np.argmax(col))            # first index of the max
            ipiv[k0 + j] = k0 + p
            piv = x[p, j]
            if p != j:
                x[[j, p], :] = x[[p, j], :]
            if piv == 0.0:
                if info == 0:
                    info = k0 + j + 1
                continue
            if j + 1 < h:
                x[j + 1:, j] = fl(x[j + 1:, j] / piv, wp)
                if j + 1 < kb:
                    l = x[j + 1:, j][:, None]
                    urow = x[j, j + 1:][None, :]
                    x[j + 1:, j + 1:] = fma_round(-l, urow, x[j + 1:, j + 1:], wp)
        # the same interchanges on the columns outside the panel
        for j in range(kb):
            r1, r2 = k0 + j, int(ipiv[k0 + j])
            if r1 != r2:
                if k0 > 0:
                    a[[r1, r2], :k0] = a[[r2, r1], :k0]
                if k0 + kb < n:
                    a[[r1, r2], k0 + kb:] = a[[r2, r1], k0 + kb:]
        a[k0:, k0:k0 + kb] = fl(x, uf)
        if k0 + kb < n:
            l11 = a[k0:k0 + kb, k0:k0 + kb]
            y = a[k0:k0 + kb, k0 + kb:].copy()
            # row r receives -l_rt * y_t for t = 0, 1, ..., r-1 in that
            # order; sweeping t outermost keeps that per-entry order
            for t in range(kb - 1):
                y[t + 1:] = fma_round(-l11[t + 1:, t][:, None], y[t][None, :],
                                      y[t + 1:], wp)
            a[k0:k0 + kb, k0 + kb:] = fl(y, uf)
            l21 = a[k0 + kb:, k0:k0 + kb]
            u12 = a[k0:k0 + kb, k0 + kb:]
            a[k0 + kb:, k0 + kb:] = fl(a[k0 + kb:, k0 + kb:] - l21 @ u12, uf)
    return LUResult(a, ipiv, info, uf)


def lu_chop(af: np.ndarray, uf: str) -> LUResult:
    """Unblocked GEPP with every operation rounded to u_f (paper mode)."""
    a = np.array(af, dtype=np.float64, copy=True)
    n = a.shape[0]
    ipiv = np.arange(n, dtype=np.int64)
    info = 0
    for j in range(n):
        p = j + int(np.argmax(np.abs(a[j:, j])))
        ipiv[j] = p
        if p != j:
            a[[j, p], :] = a[[p, j], :]
        piv = a[j, j]
        if piv == 0.0:
            if info == 0:
                info = j + 1
            continue
        if j + 1 < n:
            a[j + 1:, j] = fl(a[j + 1:, j] / piv, uf)
            prod = fl(np.outer(a[j + 1:, j], a[j, j + 1:]), uf)
            a[j + 1:, j + 1:] = fl(a[j + 1:, j + 1:] - prod, uf)
    return LUResult(a, ipiv, info, uf)
