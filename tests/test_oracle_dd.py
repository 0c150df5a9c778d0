"""Pins for the oracle's double-double path (working precision u = fp64,
u^2 = double-double, u_r = double-double): Section 3 realises the paper's
(single, double, quad) triple as (fp32, fp64, double-double) here.

Every function is compared with exact rational arithmetic
(``fractions.Fraction``) on small inputs chosen so that the low parts matter:

* the double-double operations against the relative error bounds of
  Joldes, Muller and Popescu (ACM TOMS 2017) for the accurate
  double-word + double-word sum (3u^2), double-word times double (2u^2) and
  double-word over double (3.5u^2), u = 2^-53;
* the double-double triangular solves against the forward error bound of
  substitution (Higham, ASNA Thm 8.5) with the double-double unit roundoff,
  |y - y^| <= g (|T^-1| |T| |y|), g = 2 (n + 2) 4u^2;
* the preconditioned product M^-1 v, A-tilde v (u = fp64) and the
  double-double residual b - A x against the exact value after one final
  rounding to fp64, on systems whose conditioning makes an fp64-only
  evaluation miss by many units in the last place.

The last test plants mistakes in copies of the oracle's routines (a dropped
low part, a dropped Newton correction, a wrong sign) and checks that the same
pins reject each of them.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import fp, refine

U = 2.0 ** -53
U2 = U * U


def F(x):
    return Fraction(float(x))


def dd_val(h, l):
    return F(h) + F(l)


def _rand_dd(g, size, scale_exp=20):
    """Normalised double-double values hi + lo with |lo| <= ulp(hi)/2."""
    hi = g.standard_normal(size) * np.exp2(g.integers(-scale_exp, scale_exp, size))
    lo = hi * g.uniform(-1.0, 1.0, size) * 2.0 ** -54
    hi, lo = fp.fast_two_sum(hi, lo)
    return hi, lo


def _rel_err(h, l, exact):
    if exact == 0:
        return float(abs(dd_val(h, l)))
    return float(abs(dd_val(h, l) - exact) / abs(exact))


# ---------------------------------------------------------------------------
# double-double operations
# ---------------------------------------------------------------------------

def check_dd_ops(add=None, mul=None, div=None, seed=21, count=400):
    """Largest error of each operation over its bound (<= 1 passes)."""
    add = add or fp.dd_add
    mul = mul or fp.dd_mul_d
    div = div or fp.dd_div_d
    g = np.random.default_rng(seed)
    ah, al = _rand_dd(g, count)
    bh, bl = _rand_dd(g, count)
    # half of the sums cancel heavily (b close to -a): the low parts decide
    bh[::2] = -ah[::2] * (1.0 + g.uniform(-1e-6, 1e-6, count // 2))
    bl[::2] = g.uniform(-1.0, 1.0, count // 2) * np.abs(bh[::2]) * 2.0 ** -54
    c = g.standard_normal(count) * np.exp2(g.integers(-10, 10, count))
    worst = {"add": 0.0, "mul": 0.0, "div": 0.0, "normal": 0.0}
    sh, sl = add(ah, al, bh, bl)
    ph, pl = mul(ah, al, c)
    qh, ql = div(ah, al, c)
    for i in range(count):
        a = dd_val(ah[i], al[i])
        b = dd_val(bh[i], bl[i])
        worst["add"] = max(worst["add"], _rel_err(sh[i], sl[i], a + b) / (3.0 * U2 / (1 - 4 * U)))
        worst["mul"] = max(worst["mul"], _rel_err(ph[i], pl[i], a * F(c[i])) / (2.0 * U2))
        worst["div"] = max(worst["div"], _rel_err(qh[i], ql[i], a / F(c[i])) / (3.5 * U2))
        # results are normalised: hi is the double nearest hi + lo
        for h, l in ((sh[i], sl[i]), (ph[i], pl[i]), (qh[i], ql[i])):
            if float(h) + float(l) != float(h):
                worst["normal"] = 2.0
    return worst


def test_dd_add_mul_div_within_published_bounds():
    worst = check_dd_ops()
    for name, w in worst.items():
        assert w <= 1.0, (name, w)


def test_dd_add_is_exact_when_the_sum_is_a_double_double():
    # |a| >> |b| with b a double: the exact sum is representable in two words
    a = np.array([1.0, 3.0, -7.5])
    b = np.array([2.0 ** -60, -(2.0 ** -58), 2.0 ** -70])
    h, l = fp.dd_add(a, np.zeros(3), b, np.zeros(3))
    for i in range(3):
        assert dd_val(h[i], l[i]) == F(a[i]) + F(b[i])


# ---------------------------------------------------------------------------
# triangular solves in double-double
# ---------------------------------------------------------------------------

def _exact_lower_unit(L, t):
    n = len(t)
    y = [Fraction(0)] * n
    for i in range(n):
        s = t[i]
        for j in range(i):
            s -= F(L[i, j]) * y[j]
        y[i] = s
    return y


def _exact_upper(Um, t):
    n = len(t)
    y = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        s = t[i]
        for j in range(i + 1, n):
            s -= F(Um[i, j]) * y[j]
        y[i] = s / F(Um[i, i])
    return y


def _abs_inv_abs(T, lower, unit):
    """(|T^-1| |T|) as floats, T^-1 exact."""
    n = T.shape[0]
    cols = []
    for c in range(n):
        e = [Fraction(int(i == c)) for i in range(n)]
        if lower:
            cols.append(_exact_lower_unit(T, e) if unit else None)
        else:
            cols.append(_exact_upper(T, e))
    tinv = np.array([[float(abs(cols[c][r])) for c in range(n)] for r in range(n)])
    return tinv @ np.abs(T)


def _fp16_lower_unit(g, n):
    L = np.tril(g.uniform(-1.0, 1.0, (n, n)), -1)
    L = L.astype(np.float16).astype(np.float64)
    return L + np.eye(n)


def _fp16_upper(g, n, spread=1e-3):
    Um = np.triu(g.uniform(-1.0, 1.0, (n, n)), 1)
    d = g.choice([-1.0, 1.0], n) * np.geomspace(1.0, spread, n)
    Um = Um + np.diag(d)
    return Um.astype(np.float16).astype(np.float64)


def check_dd_lower(solver=None, seed=4, n=12, trials=4):
    solver = solver or refine._dd_lower_unit
    g = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(trials):
        L = _fp16_lower_unit(g, n)
        th, tl = _rand_dd(g, n, 4)
        yh, yl = solver(L, th, tl)
        exact = _exact_lower_unit(L, [dd_val(th[i], tl[i]) for i in range(n)])
        gam = 2 * (n + 2) * 4 * U2
        bound = gam * (_abs_inv_abs(L, True, True) @ np.abs([float(v) for v in exact]))
        for i in range(n):
            err = float(abs(dd_val(yh[i], yl[i]) - exact[i]))
            worst = max(worst, err / bound[i] if bound[i] > 0 else (np.inf if err else 0))
    return worst


def check_dd_upper(solver=None, seed=6, n=12, trials=4):
    solver = solver or refine._dd_upper
    g = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(trials):
        Um = _fp16_upper(g, n)
        th, tl = _rand_dd(g, n, 4)
        yh, yl = solver(Um, th, tl)
        exact = _exact_upper(Um, [dd_val(th[i], tl[i]) for i in range(n)])
        gam = 2 * (n + 2) * 4 * U2
        bound = gam * (_abs_inv_abs(Um, False, False) @ np.abs([float(v) for v in exact]))
        for i in range(n):
            err = float(abs(dd_val(yh[i], yl[i]) - exact[i]))
            worst = max(worst, err / bound[i])
    return worst


def test_dd_lower_unit_solve_matches_exact():
    assert check_dd_lower() <= 1.0


def test_dd_upper_solve_matches_exact():
    assert check_dd_upper() <= 1.0


def test_dd_lower_solve_of_identity_is_the_input():
    th = np.array([1.0, -2.0, 3.5])
    tl = np.array([2.0 ** -60, 0.0, -(2.0 ** -55)])
    yh, yl = refine._dd_lower_unit(np.eye(3), th, tl)
    assert np.array_equal(yh, th) and np.array_equal(yl, tl)


# ---------------------------------------------------------------------------
# the preconditioned products and the residual, rounded once to fp64
# ---------------------------------------------------------------------------

def _fp64_factors(n, seed, kappa=1e10):
    """Factors of a randsvd-like matrix in u_f = fp32, u = fp64, u_r = dd."""
    g = np.random.default_rng(seed)
    q1, _ = np.linalg.qr(g.standard_normal((n, n)))
    q2, _ = np.linalg.qr(g.standard_normal((n, n)))
    a = (q1 * np.geomspace(1.0, 1.0 / kappa, n)) @ q2.T
    o = refine.Options(uf="fp32", u="fp64", ur="dd", m=10, k=0, tau=1e-8)
    return refine.factor(a, o), g


def _exact_minv(f, v):
    """2^e U^-1 L^-1 P v exactly, with the stored (rounded) factors."""
    t = [v[p] for p in f.perm]
    y = _exact_lower_unit(f.L, t)
    z = _exact_upper(f.U, y)
    return [zi * Fraction(2) ** f.e if f.e >= 0 else zi / Fraction(2) ** (-f.e) for zi in z]


def _final_rounding_excess(got, exact):
    """max over i of |got_i - exact_i| / (u |exact_i|): <= 1 means the
    double-double result was rounded correctly (up to a tie)."""
    worst = 0.0
    for gi, ei in zip(got, exact):
        err = abs(F(gi) - ei)
        worst = max(worst, float(err / (U * abs(ei))) if ei != 0 else (np.inf if err else 0.0))
    return worst


def check_minv_dd(minv=None, n=10, seed=12):
    minv = minv or refine.minv_hi
    f, g = _fp64_factors(n, seed)
    v = g.standard_normal(n)
    got = minv(f, v, "dd")
    return _final_rounding_excess(got, _exact_minv(f, [F(x) for x in v]))


def check_atilde_dd(atilde=None, n=10, seed=13):
    atilde = atilde or refine.atilde
    f, g = _fp64_factors(n, seed)
    v = g.standard_normal(n)
    got = atilde(f, v)
    av = [sum(F(f.au[i, j]) * F(v[j]) for j in range(n)) for i in range(n)]
    return _final_rounding_excess(got, _exact_minv(f, av))


def check_residual_dd(resid=None, n=12, seed=14):
    resid = resid or refine.residual
    f, g = _fp64_factors(n, seed, kappa=1e12)
    x_true = g.uniform(-1.0, 1.0, n)
    b = f.a @ x_true
    # x close to the solution: the residual cancels to ~1e-16 of |A||x|
    x = x_true + g.standard_normal(n) * 1e-13
    got = resid(f, b, x)
    exact = [F(b[i]) - sum(F(f.a[i, j]) * F(x[j]) for j in range(n)) for i in range(n)]
    # one rounding to fp64 plus the double-double sum's own n u^2 |A||x|
    worst = 0.0
    for i in range(n):
        slack = 2 * (n + 2) * 4 * U2 * float(np.abs(f.a[i]) @ np.abs(x) + abs(b[i]))
        err = float(abs(F(got[i]) - exact[i]))
        worst = max(worst, err / (U * float(abs(exact[i])) + slack))
    return worst


def test_minv_double_double_is_correctly_rounded():
    assert check_minv_dd() <= 1.0


def test_atilde_double_double_is_correctly_rounded():
    assert check_atilde_dd() <= 1.0


def test_residual_double_double_is_correctly_rounded():
    assert check_residual_dd() <= 1.0


def test_fp64_products_would_miss_these_pins():
    """The inputs are conditioned so that an evaluation in plain fp64 is off
    by many units in the last place: the pins above do see the low parts."""
    def minv64(f, v, wide):
        return refine.minv_hi(f, v, "fp64")
    assert check_minv_dd(minv64) > 4.0

    def resid64(f, b, x):
        return b - f.a @ x
    assert check_residual_dd(resid64) > 4.0


def test_dd_gemv_offset_and_sign():
    g = np.random.default_rng(15)
    a = g.standard_normal((5, 17))
    x = g.standard_normal(17)
    y0h, y0l = _rand_dd(g, 5, 2)
    for sign in (1.0, -1.0):
        hi, lo = fp.dd_gemv(a, x, y0h=y0h, y0l=y0l, sign=sign)
        for i in range(5):
            ex = dd_val(y0h[i], y0l[i]) + Fraction(int(sign)) * sum(
                F(a[i, j]) * F(x[j]) for j in range(17))
            err = float(abs(dd_val(hi[i], lo[i]) - ex))
            assert err <= 2 * 19 * 4 * U2 * (float(np.abs(a[i]) @ np.abs(x)) + abs(y0h[i]))


# ---------------------------------------------------------------------------
# planted mistakes: each must be rejected by at least one pin above
# ---------------------------------------------------------------------------

def _add_drop_low(ah, al, bh, bl):
    return fp.two_sum(ah, bh)


def _mul_drop_low(ah, al, b):
    p, e = fp.two_prod(ah, b)
    return fp.fast_two_sum(p, e)


def _div_no_correction(ah, al, b):
    return ah / b, np.zeros_like(np.asarray(ah / b))


def _lower_drop_yl(L, th, tl):
    n = L.shape[0]
    yh, yl = th.copy(), tl.copy()
    for j in range(n - 1):
        col = L[j + 1:, j]
        p, e = fp.two_prod(col, yh[j])
        yh[j + 1:], yl[j + 1:] = fp.dd_add(yh[j + 1:], yl[j + 1:], -p, -e)
    return yh, yl


def _upper_wrong_index(Um, th, tl):
    n = Um.shape[0]
    yh, yl = th.copy(), tl.copy()
    for j in range(n - 1, -1, -1):
        qh, ql = fp.dd_div_d(yh[j], yl[j], Um[j, j])
        yh[j], yl[j] = qh, ql
        if j > 0:
            col = Um[j, :j]          # a row where the column belongs
            p, e = fp.two_prod(col, qh)
            e = e + col * ql
            yh[:j], yl[:j] = fp.dd_add(yh[:j], yl[:j], -p, -e)
    return yh, yl


def _residual_wrong_sign(f, b, x):
    rh, rl = fp.dd_gemv(f.a, x, y0h=b, y0l=np.zeros_like(b), sign=1.0)
    return rh + rl


def test_planted_mistakes_are_caught(monkeypatch):
    assert check_dd_ops(add=_add_drop_low)["add"] > 1.0
    assert check_dd_ops(mul=_mul_drop_low)["mul"] > 1.0
    assert check_dd_ops(div=_div_no_correction)["div"] > 1.0
    assert check_dd_lower(_lower_drop_yl) > 1.0
    assert check_dd_upper(_upper_wrong_index) > 1.0
    assert check_residual_dd(_residual_wrong_sign) > 1.0
    # the same mistakes reached through the oracle's own entry points
    with monkeypatch.context() as mp:
        mp.setattr(fp, "dd_add", _add_drop_low)
        assert check_minv_dd() > 1.0
    with monkeypatch.context() as mp:
        mp.setattr(fp, "dd_div_d", _div_no_correction)
        assert check_atilde_dd() > 1.0
    with monkeypatch.context() as mp:
        mp.setattr(refine, "_dd_lower_unit", _lower_drop_yl)
        assert check_atilde_dd() > 1.0


# ---------------------------------------------------------------------------
# Table tab:prec_gmresIR: inside the printed kappa_inf limit GMRES-IR converges
# ---------------------------------------------------------------------------

def _randsvd(n, kappa, seed):
    g = np.random.default_rng(seed)
    q1, r1 = np.linalg.qr(g.standard_normal((n, n)))
    q1 = q1 * np.sign(np.diag(r1))
    q2, r2 = np.linalg.qr(g.standard_normal((n, n)))
    q2 = q2 * np.sign(np.diag(r2))
    a = (q1 * np.geomspace(1.0, 1.0 / kappa, n)) @ q2.T
    x = g.uniform(-1.0, 1.0, n)
    return a, x, a @ x


# the oracle's precision names for the table's rows (quad -> double-double);
# rows with u = fp16 have no counterpart here (u is fp32 or fp64)
_ROW_MAP = {"fp16": "fp16", "fp32": "fp32", "fp64": "fp64", "fp128": "dd"}


def test_table_prec_gmresir_limits_converge(golden_dir):
    with open(os.path.join(golden_dir, "tab_prec_gmresir.json")) as fh:
        rows = json.load(fh)["rows"]
    ran = 0
    n = 48
    for row in rows:
        if row["u"] == "fp16":
            continue
        uf, u, ur = (_ROW_MAP[row[k]] for k in ("uf", "u", "ur"))
        # kappa_2 two decades inside the printed kappa_inf limit
        kappa2 = row["kappa_inf"] / 100.0
        a, x_true, b = _randsvd(n, kappa2, 3)
        kinf = np.linalg.norm(a, np.inf) * np.linalg.norm(np.linalg.inv(a), np.inf)
        assert kinf < row["kappa_inf"], (row, kinf)
        tau = 1e-4 if u == "fp32" else 1e-8
        o = refine.Options(uf=uf, u=u, ur=ur, m=n, k=0, tau=tau, imax=10, berr_target=1e-15)
        x, info, _ = refine.gmresir(a, b, o)
        assert info.status == refine.STATUS_OK, (row, info.berr)
        # Table 2's limiting errors: backward error of order u_x = fp64 and a
        # forward error of order kappa_inf u_x
        assert info.berr[-1] <= 1e-15
        ferr = np.max(np.abs(x - x_true)) / np.max(np.abs(x_true))
        assert ferr <= 10 * kinf * U
        ran += 1
    assert ran == 4
