"""Pins for the oracle's precision emulation (rounding and double-double).

The rounding routines are pinned to the unit roundoffs printed in the paper
(Table "tab:eps"), to exhaustive round trips of every fp16/bf16 bit pattern,
to two independent rounding implementations agreeing, and to exact rational
arithmetic for the error-free transformations.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import fp


def test_unit_roundoffs_match_paper_table(golden_dir):
    with open(os.path.join(golden_dir, "tab_eps.json")) as fh:
        tab = json.load(fh)["unit_roundoff"]
    for name, printed in tab.items():
        mine = fp.FORMATS[name].unit_roundoff
        assert abs(mine - printed) / printed < 5e-3, (name, mine, printed)
    # and they are exactly the powers of two 2^-p
    assert fp.unit_roundoff("fp16") == 2.0 ** -11
    assert fp.unit_roundoff("fp32") == 2.0 ** -24
    assert fp.unit_roundoff("fp64") == 2.0 ** -53
    assert fp.unit_roundoff("bf16") == 2.0 ** -8


def _all_fp16():
    bits = np.arange(1 << 16, dtype=np.uint16)
    v = bits.view(np.float16).astype(np.float64)
    return v[np.isfinite(v)]


def _all_bf16():
    bits = (np.arange(1 << 16, dtype=np.uint32) << 16).astype(np.uint32)
    v = bits.view(np.float32).astype(np.float64)
    return v[np.isfinite(v)]


def test_fp16_every_pattern_round_trips():
    v = _all_fp16()
    assert np.array_equal(fp.fl(v, "fp16"), v)
    assert np.array_equal(fp.round_to_format(v, fp.FP16), v)


def test_bf16_every_pattern_round_trips():
    v = _all_bf16()
    assert np.array_equal(fp.fl(v, "bf16"), v)


def _midpoints(sorted_vals):
    pos = sorted_vals[sorted_vals > 0]
    pos = np.unique(pos)
    return pos[:-1], pos[1:], 0.5 * (pos[:-1] + pos[1:])


def _is_even_fp16(x):
    bits = x.astype(np.float16).view(np.uint16)
    return (bits & 1) == 0


def test_fp16_ties_round_to_even():
    lo, hi, mid = _midpoints(_all_fp16())
    got = fp.round_to_format(mid, fp.FP16)
    want = np.where(_is_even_fp16(lo), lo, hi)
    assert np.array_equal(got, want)
    assert np.array_equal(fp.fl(mid, "fp16"), want)


def test_bf16_ties_round_to_even():
    lo, hi, mid = _midpoints(_all_bf16())
    got = fp.fl(mid, "bf16")
    lo_bits = (lo.astype(np.float32).view(np.uint32) >> 16) & 1
    want = np.where(lo_bits == 0, lo, hi)
    assert np.array_equal(got, want)


def _bf16_from_fp32_bits(x32):
    """Independent integer rounding of fp32 values to bf16 (RNE)."""
    b = x32.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_matches_integer_rounding_on_fp32_inputs():
    g = np.random.default_rng(7)
    x = (g.standard_normal(200000) * np.exp2(g.integers(-140, 120, 200000))).astype(np.float32)
    got = fp.fl(x.astype(np.float64), "bf16")
    want = _bf16_from_fp32_bits(x)
    ok = np.isfinite(want)
    assert np.array_equal(got[ok], want[ok])


def test_generic_rounding_matches_numpy_casts():
    g = np.random.default_rng(3)
    x = g.standard_normal(100000) * np.exp2(g.integers(-160, 140, 100000))
    assert np.array_equal(fp.round_to_format(x, fp.FP32), x.astype(np.float32).astype(np.float64))
    y = g.standard_normal(100000) * np.exp2(g.integers(-30, 20, 100000))
    assert np.array_equal(fp.round_to_format(y, fp.FP16), y.astype(np.float16).astype(np.float64))


def test_overflow_and_underflow():
    assert fp.fl(np.array([70000.0]), "fp16")[0] == np.inf
    assert fp.fl(np.array([65519.0]), "fp16")[0] == 65504.0
    assert fp.fl(np.array([2.0 ** -26]), "fp16")[0] == 0.0   # below half the min subnormal
    big = 2.0 ** 128
    assert fp.fl(np.array([big]), "bf16")[0] == np.inf


def _frac(x):
    return Fraction(float(x))


def test_two_sum_and_two_prod_are_exact():
    g = np.random.default_rng(11)
    a = g.standard_normal(2000) * np.exp2(g.integers(-40, 40, 2000))
    b = g.standard_normal(2000) * np.exp2(g.integers(-40, 40, 2000))
    s, e = fp.two_sum(a, b)
    p, f = fp.two_prod(a, b)
    for i in range(0, 2000, 37):
        assert _frac(s[i]) + _frac(e[i]) == _frac(a[i]) + _frac(b[i])
        assert _frac(p[i]) + _frac(f[i]) == _frac(a[i]) * _frac(b[i])


def test_dot2_within_ogita_rump_oishi_bound():
    g = np.random.default_rng(5)
    u = 2.0 ** -53
    for n in (3, 10, 50, 200):
        for _ in range(5):
            x = g.standard_normal(n) * np.exp2(g.integers(-20, 20, n))
            y = g.standard_normal(n)
            y[-1] = -float(sum(_frac(xi) * _frac(yi) for xi, yi in zip(x[:-1], y[:-1])) / _frac(x[-1]))
            exact = sum(_frac(xi) * _frac(yi) for xi, yi in zip(x, y))
            got = fp.dot2(x, y)
            gam = n * u / (1 - n * u)
            bound = u * abs(float(exact)) + gam * gam * float(np.sum(np.abs(x * y)))
            assert abs(float(_frac(got) - exact)) <= bound * 1.0001 + 1e-300


def test_dd_gemv_matches_exact_products():
    g = np.random.default_rng(9)
    a = g.standard_normal((6, 40))
    x = g.standard_normal(40)
    hi, lo = fp.dd_gemv(a, x)
    for i in range(6):
        exact = sum(_frac(a[i, j]) * _frac(x[j]) for j in range(40))
        err = abs(_frac(hi[i]) + _frac(lo[i]) - exact)
        assert float(err) <= 1e-30 * max(1.0, abs(float(exact))) + 40 * 2.0 ** -104 * float(np.abs(a[i] * x).sum())


def test_square_precision_map():
    assert fp.square_precision("fp32") == "fp64"
    assert fp.square_precision("fp64") == "dd"
    assert fp.square_precision("fp16") == "fp32"
