"""Pins for the oracle's GEPP in u_f.

* brute force: a textbook unblocked GEPP in exact rational arithmetic (written
  here, independently) gives the same pivots and, in fp64 mode, the same
  factors to rounding level; its own factors satisfy P A = L U exactly;
* LAPACK (scipy.linalg.lu_factor) chooses the same pivot rows on random
  matrices;
* the low-precision factors satisfy the componentwise backward-error bound
  |P A - L U| <= c u_f |L| |U| (Higham, Accuracy and Stability of Numerical
  Algorithms, Thm 9.3, with one u_f rounding per block step);
* A = I factors to I; a zero column reports the singular column;
* the fused multiply-add emulation is correctly rounded (checked against
  exact rational rounding).
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fp
from oracle.lu import (fma_round, fp16_scale_exponent, lu_blocked, lu_chop,
                       perm_from_ipiv, unpack)
from synthetic import randsvd


def exact_gepp(a):
    """Unblocked GEPP over the rationals; pivot = first row of max |a|."""
    n = len(a)
    m = [[Fraction(x) for x in row] for row in a]
    piv = list(range(n))
    for j in range(n):
        p = max(range(j, n), key=lambda i: (abs(m[i][j]), -i))
        piv[j] = p
        m[j], m[p] = m[p], m[j]
        if m[j][j] == 0:
            continue
        for i in range(j + 1, n):
            m[i][j] = m[i][j] / m[j][j]
            for c in range(j + 1, n):
                m[i][c] -= m[i][j] * m[j][c]
    return m, piv


def _perm(piv):
    p = list(range(len(piv)))
    for i, j in enumerate(piv):
        p[i], p[j] = p[j], p[i]
    return p


@pytest.mark.parametrize("seed", range(6))
def test_exact_rational_gepp_reconstructs_and_matches(seed):
    g = np.random.default_rng(seed)
    n = 7
    a = g.integers(-9, 10, size=(n, n)).astype(np.float64)
    if abs(np.linalg.det(a)) < 0.5:
        a[np.diag_indices(n)] += 20
    m, piv = exact_gepp(a.tolist())
    # the brute force itself: P A = L U exactly
    perm = _perm(piv)
    for i in range(n):
        for c in range(n):
            s = sum((m[i][t] if t < i else (1 if t == i else 0)) * (m[t][c] if t <= c else 0)
                    for t in range(n))
            assert s == Fraction(int(a[perm[i], c]))
    # the oracle, fp64 storage, several block sizes
    for nb in (1, 2, 3, 7):
        res = lu_blocked(a, "fp64", nb)
        assert list(res.ipiv) == piv
        exact = np.array([[float(x) for x in row] for row in m])
        assert np.allclose(res.lu, exact, rtol=1e-13, atol=1e-13)


def test_pivots_match_lapack():
    g = np.random.default_rng(1)
    for n, nb in ((50, 8), (64, 16), (97, 32)):
        a = g.standard_normal((n, n))
        res = lu_blocked(a, "fp64", nb)
        _, piv = sla.lu_factor(a)
        assert np.array_equal(res.ipiv, piv)
        L, U = unpack(res.lu)
        assert np.abs(a[res.perm] - L @ U).max() < 1e-12


def test_identity_and_permutation():
    for uf in ("fp16", "bf16", "fp32"):
        res = lu_blocked(np.eye(9), uf, 4)
        assert np.array_equal(res.lu, np.eye(9))
        assert np.array_equal(res.ipiv, np.arange(9))
    p = np.eye(5)[[3, 0, 4, 1, 2]]
    res = lu_blocked(p, "fp16", 2)
    assert np.array_equal(p[res.perm], np.eye(5))


def test_perm_from_ipiv_applies_swaps_in_order():
    ipiv = np.array([2, 2, 3, 3])
    perm = perm_from_ipiv(ipiv)
    b = np.arange(4.0)
    c = b.copy()
    for i, j in enumerate(ipiv):
        c[[i, j]] = c[[j, i]]
    assert np.array_equal(b[perm], c)


@pytest.mark.parametrize("uf,nb", [("fp16", 16), ("fp16", 64), ("bf16", 32), ("fp32", 16)])
def test_componentwise_backward_error_bound(uf, nb):
    n = 192
    a = randsvd(n, 1e4, 3)
    e = fp16_scale_exponent(np.abs(a).max(), n) if uf == "fp16" else 0
    af = fp.fl(np.ldexp(a, e), uf)
    res = lu_blocked(af, uf, nb)
    assert res.info == 0
    L, U = unpack(res.lu)
    lhs = np.abs(af[res.perm] - L @ U)
    rhs = np.abs(L) @ np.abs(U)
    c = 2 * (n // nb + 3) * fp.unit_roundoff(uf)
    assert np.all(lhs <= c * rhs + 1e-300)
    # and the bound is not vacuous: errors are of order u_f somewhere
    assert lhs.max() > 0


def test_paper_mode_backward_error_bound():
    n = 60
    a = randsvd(n, 1e3, 2)
    af = fp.fl(np.ldexp(a, fp16_scale_exponent(np.abs(a).max(), n)), "fp16")
    res = lu_chop(af, "fp16")
    L, U = unpack(res.lu)
    lhs = np.abs(af[res.perm] - L @ U)
    gam = n * fp.unit_roundoff("fp16") / (1 - n * fp.unit_roundoff("fp16"))
    assert np.all(lhs <= 2 * gam * (np.abs(L) @ np.abs(U)))


def test_singular_column_reported():
    a = np.random.default_rng(0).standard_normal((12, 12))
    a[:, 5] = 0.0
    res = lu_blocked(a, "fp32", 4)
    assert res.info == 6


def test_scale_exponent():
    for n in (1, 100, 8192):
        for amax in (1e-3, 0.5, 1.0, 3.0, 4094.0, 5000.0, 1e-30):
            e = fp16_scale_exponent(amax, n)
            t = amax * np.sqrt(n)
            assert np.ldexp(t, e) <= 4094.0 < np.ldexp(t, e + 1)


def _round_fraction_to_fp32(q):
    """Round a Fraction to the nearest fp32 (ties to even) by exhaustion of
    the two neighbours."""
    f = np.float32(float(q))              # within one ulp
    cands = [f, np.nextafter(f, np.float32(np.inf)), np.nextafter(f, np.float32(-np.inf))]
    best = min(cands, key=lambda c: (abs(Fraction(float(c)) - q),
                                     int(np.array(c).view(np.uint32)) & 1))
    return float(best)


def test_fma_emulation_is_correctly_rounded():
    g = np.random.default_rng(4)
    a = g.standard_normal(3000).astype(np.float32).astype(np.float64)
    b = g.standard_normal(3000).astype(np.float32).astype(np.float64)
    c = (-(a * b) * (1 + g.standard_normal(3000) * 1e-6)).astype(np.float32).astype(np.float64)
    got = fma_round(a, b, c, "fp32")
    for i in range(0, 3000, 7):
        q = Fraction(a[i]) * Fraction(b[i]) + Fraction(c[i])
        assert got[i] == _round_fraction_to_fp32(q), i
