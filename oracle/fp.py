"""Precision emulation for the oracle (test infrastructure only).

The paper simulates half precision with the ``chop`` library and quadruple
precision with a multiprecision toolbox (Section 3).  Here every low-precision
value is held in a float64 array and rounded to its format with
round-to-nearest-even, subnormals kept:

* fp16 and fp32 use numpy's direct float64 -> float16/float32 conversions;
* bf16 (8-bit significand, fp32 exponent range) and any other binary format
  use :func:`round_to_format`, which scales by the value's ulp and rounds
  with numpy's half-to-even ``rint``;
* "double-double" (the u^2 of an fp64 working precision) is built from
  error-free transformations: Knuth's TwoSum, Dekker's TwoProduct with
  Veltkamp splitting (Python 3.10 has no fused multiply-add), and the
  compensated dot product Dot2 of Ogita, Rump and Oishi (2005).

Unit roundoffs (Table "tab:eps" of the paper): fp16 2^-11 = 4.88e-4,
fp32 2^-24 = 5.96e-8, fp64 2^-53 = 1.11e-16, fp128 2^-113 = 9.63e-35;
bf16 has 2^-8 (not in the paper).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Format:
    """A binary floating-point format: significand bits p (including the
    implicit bit), minimum normal exponent emin, maximum exponent emax."""
    name: str
    p: int
    emin: int
    emax: int

    @property
    def unit_roundoff(self) -> float:
        return math.ldexp(1.0, -self.p)

    @property
    def max_finite(self) -> float:
        return math.ldexp(2.0 - math.ldexp(1.0, 1 - self.p), self.emax)

    @property
    def min_normal(self) -> float:
        return math.ldexp(1.0, self.emin)


FP16 = Format("fp16", 11, -14, 15)
BF16 = Format("bf16", 8, -126, 127)
FP32 = Format("fp32", 24, -126, 127)
FP64 = Format("fp64", 53, -1022, 1023)
FP128 = Format("fp128", 113, -16382, 16383)

FORMATS = {f.name: f for f in (FP16, BF16, FP32, FP64, FP128)}

# precision names accepted by the solver options; "dd" is double-double
PRECISIONS = ("fp16", "bf16", "fp32", "fp64", "dd")


def unit_roundoff(prec: str) -> float:
    if prec == "dd":
        return math.ldexp(1.0, -104)
    return FORMATS[prec].unit_roundoff


def square_precision(u: str) -> str:
    """The precision u^2 in which Alg. 2/3 apply the preconditioned matrix:
    fp16 -> fp32, fp32 -> fp64, fp64 -> double-double."""
    return {"fp16": "fp32", "bf16": "fp32", "fp32": "fp64", "fp64": "dd"}[u]


def round_to_format(x, fmt: Format) -> np.ndarray:
    """Round float64 values to ``fmt`` (nearest, ties to even), returned as
    float64.  Overflow gives +-inf, values below the subnormal range flush to
    signed zero.  Independent of numpy's float16/float32 casts."""
    x = np.asarray(x, dtype=np.float64)
    out = np.array(x, copy=True)
    finite = np.isfinite(x) & (x != 0)
    if not np.any(finite):
        return out
    xf = x[finite]
    _, e = np.frexp(xf)                  # |x| = m 2^e, m in [0.5, 1)
    e = e - 1                            # |x| = m' 2^e, m' in [1, 2)
    e = np.maximum(e, fmt.emin)          # subnormal spacing below emin
    shift = (fmt.p - 1) - e              # ulp = 2^(e - p + 1)
    q = np.rint(np.ldexp(xf, shift))     # exact scaling, half-to-even
    r = np.ldexp(q, -shift)
    r = np.where(np.abs(r) > fmt.max_finite, np.copysign(np.inf, xf), r)
    r = np.where(r == 0, np.copysign(0.0, xf), r)
    out[finite] = r
    return out


def fl(x, prec: str) -> np.ndarray:
    """Round to precision ``prec`` and return float64 values."""
    x = np.asarray(x, dtype=np.float64)
    if prec == "fp16":
        return x.astype(np.float16).astype(np.float64)
    if prec == "fp32":
        return x.astype(np.float32).astype(np.float64)
    if prec == "bf16":
        return round_to_format(x, BF16)
    if prec in ("fp64", "dd"):
        return np.array(x, dtype=np.float64, copy=True)
    raise ValueError(f"unknown precision {prec!r}")


def fl32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# error-free transformations and double-double arithmetic
# --------------------------------------------------------------------------

_SPLITTER = 134217729.0  # 2^27 + 1 (Veltkamp splitting for binary64)


def two_sum(a, b):
    """Knuth's TwoSum: s + e == a + b exactly, s = fl(a + b)."""
    s = a + b
    bb = s - a
    e = (a - (s - bb)) + (b - bb)
    return s, e


def fast_two_sum(a, b):
    """Dekker's FastTwoSum; requires |a| >= |b| (or a == 0)."""
    s = a + b
    e = b - (s - a)
    return s, e


def split(a):
    """Veltkamp splitting a = hi + lo with 26-bit halves."""
    c = _SPLITTER * a
    hi = c - (c - a)
    lo = a - hi
    return hi, lo


def two_prod(a, b):
    """Dekker's TwoProduct: p + e == a * b exactly (no overflow assumed)."""
    p = a * b
    ah, al = split(a)
    bh, bl = split(b)
    e = al * bl - (((p - ah * bh) - al * bh) - ah * bl)
    return p, e


def dd_add(ah, al, bh, bl):
    """Double-double + double-double (accurate variant)."""
    s, e = two_sum(ah, bh)
    t, f = two_sum(al, bl)
    e = e + t
    s, e = fast_two_sum(s, e)
    e = e + f
    return fast_two_sum(s, e)


def dd_mul_d(ah, al, b):
    """Double-double times double."""
    p, e = two_prod(ah, b)
    e = e + al * b
    return fast_two_sum(p, e)


def dd_div_d(ah, al, b):
    """Double-double divided by double (one Newton correction)."""
    q1 = ah / b
    p, e = two_prod(q1, b)
    r = ((ah - p) - e) + al
    q2 = r / b
    return fast_two_sum(q1, q2)


def dot2(x, y):
    """Ogita-Rump-Oishi Dot2: fl(x . y) computed as if in twice the working
    precision, then rounded once.  Returns a float64 scalar."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.size == 0:
        return 0.0
    p, s = two_prod(x[0], y[0])
    for i in range(1, x.size):
        h, r = two_prod(x[i], y[i])
        p, q = two_sum(p, h)
        s = s + (q + r)
    return float(p + s)


def dd_gemv(a, x, y0h=None, y0l=None, sign=1.0):
    """Row-wise compensated matrix-vector product in double-double.

    Returns (hi, lo) with hi + lo ~= y0 + sign * (A x), each row accumulated
    with TwoProduct/TwoSum (a vectorised Dot2 that keeps the low part).
    """
    a = np.asarray(a, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    m = a.shape[0]
    hi = np.zeros(m) if y0h is None else np.array(y0h, dtype=np.float64)
    lo = np.zeros(m) if y0l is None else np.array(y0l, dtype=np.float64)
    for j in range(a.shape[1]):
        p, e = two_prod(a[:, j], sign * x[j])
        hi, q = two_sum(hi, p)
        lo = lo + (q + e)
    return fast_two_sum(hi, lo)
