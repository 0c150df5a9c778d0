"""Pins for the oracle's adjoint solve (A^T lambda = g with the transposed
factors) and the gradient of a loss through x = A^-1 b.

* M^-T from the factors equals the inverse transpose of the explicitly
  assembled M = 2^-e P^T L U (and M^-1 its inverse), with pivoting that
  moves rows (brute force at small n);
* adjoint identities u^T (M^-1 v) = (M^-T u)^T v and
  u^T (A_u M^-1 v) = (M^-T A_u^T u)^T v;
* the transposed refinement reaches the backward-error target for A^T and
  agrees with a dense fp64 solve of A^T lambda = g to kappa u;
* the gradient dL/dA = -lambda x^T, dL/db = lambda of L = 0.5 ||x - y||^2
  matches central finite differences (n = 64) and the dense fp64 gradient.
"""
import numpy as np
import pytest

from oracle import Options, factor, refine, solve
from synthetic import randsvd_problem

U64 = 2.0 ** -53


def _opts(**kw):
    base = dict(uf="fp16", u="fp32", ur="fp64", m=20, k=5, tau=1e-4, nb=16)
    base.update(kw)
    return Options(**base)


def _assembled_m(f):
    """M = 2^-e P^T L U as a dense matrix (P b = b[perm])."""
    lu = f.L @ f.U
    m = np.empty_like(lu)
    m[f.perm] = lu
    return np.ldexp(m, -f.e)


@pytest.mark.parametrize("uf", ["fp16", "fp32"])
def test_minv_t_is_inverse_transpose_of_assembled_m(uf):
    g = np.random.default_rng(3)
    a = g.standard_normal((30, 30))
    f = factor(a, _opts(uf=uf))
    assert np.any(f.perm != np.arange(30))          # rows really move
    mm = _assembled_m(f)
    v = g.standard_normal(30)
    ref_t = np.linalg.solve(mm.T, v)
    ref = np.linalg.solve(mm, v)
    assert np.allclose(refine.minv_t(f, v), ref_t, rtol=1e-10, atol=1e-12 * np.abs(ref_t).max())
    assert np.allclose(refine.minv_hi(f, v, "fp64"), ref, rtol=1e-10,
                       atol=1e-12 * np.abs(ref).max())


def test_adjoint_identities():
    p = randsvd_problem(70, 1e4, 5)
    f = factor(p.a, _opts())
    g = np.random.default_rng(9)
    u, v = g.standard_normal(70), g.standard_normal(70)
    lhs = u @ refine.minv_hi(f, v, "fp64")
    rhs = refine.minv_t(f, u) @ v
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    # the adjoint's operator M^-T A_u^T is the transpose of A_u M^-1
    lhs = u @ (f.au @ refine.minv_hi(f, v, "fp64"))
    rhs = refine.minv_t(f, f.au.T @ u) @ v
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


@pytest.mark.parametrize("k", [5, 0])
def test_transposed_refinement_converges(k):
    p = randsvd_problem(100, 1e4, 2)
    f = factor(p.a, _opts(k=k))
    gvec = np.random.default_rng(1).standard_normal(100)
    lam, info = refine.solve_transposed(f, gvec)
    assert info.status == refine.STATUS_OK
    r = gvec - p.a.T @ lam
    norm_a1 = np.max(np.sum(np.abs(p.a), axis=0))
    eta = np.max(np.abs(r)) / (norm_a1 * np.max(np.abs(lam)) + np.max(np.abs(gvec)))
    assert eta <= 1e-14
    assert abs(eta - info.berr[-1]) <= 1e-3 * max(eta, 1e-30) + 1e-30
    ref = np.linalg.solve(p.a.T, gvec)
    kappa = np.linalg.cond(p.a, np.inf)
    assert np.max(np.abs(lam - ref)) / np.max(np.abs(ref)) <= 10 * kappa * 100 * U64


def _loss(a, b, y):
    x = np.linalg.solve(a, b)
    return 0.5 * float(np.sum((x - y) ** 2))


def test_gradient_matches_finite_differences_and_dense_reference():
    n = 64
    p = randsvd_problem(n, 1e3, 4)
    rng = np.random.default_rng(11)
    y = rng.standard_normal(n)
    f = factor(p.a, _opts(k=3, m=10))
    x, info = solve(f, p.b)
    assert info.status == refine.STATUS_OK
    da, db, ainfo = refine.gradient(f, x, x - y)
    assert ainfo.status == refine.STATUS_OK
    # dense fp64 reference
    xr = np.linalg.solve(p.a, p.b)
    lr = np.linalg.solve(p.a.T, xr - y)
    assert np.max(np.abs(da + np.outer(lr, xr))) <= 1e-9 * np.max(np.abs(np.outer(lr, xr)))
    assert np.max(np.abs(db - lr)) <= 1e-9 * np.max(np.abs(lr))
    # central differences along random directions
    h = 1e-8
    for _ in range(3):
        e_a = rng.standard_normal((n, n))
        e_b = rng.standard_normal(n)
        fd = (_loss(p.a + h * e_a, p.b + h * e_b, y)
              - _loss(p.a - h * e_a, p.b - h * e_b, y)) / (2 * h)
        an = float(np.sum(da * e_a) + db @ e_b)
        assert abs(fd - an) <= 1e-5 * abs(an)


def test_transposed_solve_rejects_other_triples():
    p = randsvd_problem(30, 1e2, 1)
    f = factor(p.a, _opts(uf="fp32", u="fp64", ur="dd"))
    with pytest.raises(ValueError):
        refine.solve_transposed(f, p.b)


def test_choose_k_matches_brute_force_runs():
    """The sweep's iteration counts are those of independent runs with each
    k (the factorisation does not depend on k), and the chosen k is the
    smallest one attaining the minimum below the first-step limit."""
    from oracle import gmresir
    p = randsvd_problem(100, 1e4, 3)
    o = _opts(m=20, k=8)
    f = factor(p.a, o)
    kb, its = refine.choose_k(f, p.b, 8)
    x0, info0, _ = gmresir(p.a, p.b, _opts(m=20, k=0))
    limit = info0.its[0] - 1
    for k in range(9):
        if k > limit:
            assert its[k] == -1
            continue
        _, info, _ = gmresir(p.a, p.b, _opts(m=20, k=k))
        assert its[k] == (info.total_its if info.status == refine.STATUS_OK else -1)
    valid = [(t, k) for k, t in enumerate(its) if t >= 0]
    assert kb == min(valid)[1]
    assert kb <= limit
