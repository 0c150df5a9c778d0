"""Pins for the oracle's GMRES / GCRO-DR (Section 2 of the paper).

Solver-level checks pass the operator directly (no LU), so each fact is a
property of the Krylov method alone:

* the Givens least-squares solution equals numpy's lstsq on the same Hbar;
* A = I converges in one iteration for any right-hand side;
* an operator with d distinct eigenvalues converges in exactly d steps in
  fp64 (degree of the minimal polynomial);
* the Arnoldi relation A V_j = V_{j+1} Hbar_j (+ C B) holds to rounding level;
* the first-cycle harmonic Ritz form of the algorithm equals the generalised
  form Hbar^T Hbar z = theta H^T z, and reduces to eig(H) on an invariant
  subspace;
* GCRO-DR with k = 0 reproduces an independent textbook restarted GMRES;
* after a refresh, A U_k = C_k and C_k^T C_k = I hold to rounding level;
* exact deflation: with U_k spanning an invariant subspace of the small
  eigenvalues, the recycled solve needs 1 iteration against d + 1;
* recycling does not change the first refinement step (Section 3).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import krylov
from oracle.krylov import KrylovOptions, RecycleState, gcrodr


def _same_spectrum(a, b, rtol):
    a = np.asarray(a, dtype=complex)
    b = list(np.asarray(b, dtype=complex))
    assert len(a) == len(b)
    for x in a:
        i = int(np.argmin([abs(x - y) for y in b]))
        assert abs(x - b[i]) <= rtol * max(1.0, abs(x)), (x, b[i])
        b.pop(i)


def _ops(mat, u="fp64"):
    from oracle.fp import fl
    return (lambda v: fl(mat @ v, u)), (lambda y: mat @ y)


def test_givens_matches_lstsq():
    g = np.random.default_rng(0)
    for j in (1, 3, 10, 25):
        h = np.triu(g.standard_normal((j + 1, j)), -1)
        beta = 2.5
        y, est = krylov.givens_lsq(h, beta)
        c = np.zeros(j + 1)
        c[0] = beta
        y_ref, *_ = np.linalg.lstsq(h, c, rcond=None)
        assert np.allclose(y, y_ref, rtol=1e-10, atol=1e-12)
        assert abs(est - np.linalg.norm(c - h @ y_ref)) < 1e-10 * beta


@pytest.mark.parametrize("u", ["fp32", "fp64"])
def test_identity_converges_in_one_iteration(u):
    g = np.random.default_rng(1)
    n = 50
    ap, a64 = _ops(np.eye(n), u)
    for k in (0, 3):
        z = g.standard_normal(n)
        d, rec = gcrodr(ap, a64, z, KrylovOptions(m=10, k=k, tau=1e-4, u=u), RecycleState())
        assert rec.its == 1
        assert np.allclose(d, z, rtol=1e-6)


@pytest.mark.parametrize("ndist", [1, 2, 5, 9])
def test_distinct_eigenvalues_give_exact_count(ndist):
    g = np.random.default_rng(ndist)
    n = 60
    vals = np.linspace(1.0, 3.0, ndist)
    diag = vals[g.integers(0, ndist, n)]
    diag[:ndist] = vals                   # every value present
    s = sla.qr(g.standard_normal((n, n)))[0]
    mat = s @ np.diag(diag) @ s.T         # normal, ndist distinct eigenvalues
    ap, a64 = _ops(mat)
    z = g.standard_normal(n)
    d, rec = gcrodr(ap, a64, z, KrylovOptions(m=20, k=0, tau=1e-10, u="fp64"), RecycleState())
    assert rec.its == ndist
    assert np.linalg.norm(mat @ d - z) <= 1e-9 * np.linalg.norm(z)


def test_arnoldi_relation_with_projection():
    g = np.random.default_rng(3)
    n, j, kc = 80, 12, 3
    mat = g.standard_normal((n, n)) / np.sqrt(n) + 2 * np.eye(n)
    C = sla.qr(g.standard_normal((n, kc)), mode="economic")[0]
    ap, _ = _ops(mat, "fp32")
    r = g.standard_normal(n)
    r = r - C @ (C.T @ r)
    opts = KrylovOptions(m=40, k=kc, tau=1e-30, u="fp32")
    V, Hb, B, jj, gv, beta, est = krylov._arnoldi(ap, r, C, j, 0.0, opts)
    assert jj == j
    lhs = mat @ V[:, :j]
    rhs = C @ B + V @ Hb
    u32 = 2.0 ** -24
    assert np.linalg.norm(lhs - rhs) <= 10 * j * n * u32 * np.linalg.norm(mat, 2)
    assert np.linalg.norm(V.T @ V - np.eye(j + 1)) < 1e-5
    assert np.linalg.norm(C.T @ V) < 1e-5


def test_harmonic_ritz_first_equals_generalised_form():
    g = np.random.default_rng(4)
    j = 12
    hb = np.triu(g.standard_normal((j + 1, j)), -1) + 3 * np.eye(j + 1, j)
    hm = hb[:j]
    theta_g = sla.eig(hb.T @ hb, hm.T, right=False)
    ej = np.zeros(j)
    ej[-1] = 1
    f = np.linalg.solve(hm.T, ej)
    mat = hm.copy()
    mat[:, -1] += hb[j, j - 1] ** 2 * f
    theta_p = np.linalg.eigvals(mat)
    _same_spectrum(theta_g, theta_p, 1e-8)
    # the oracle's general routine with W^T V = [I; 0] spans the same space
    p1 = krylov.harmonic_ritz_first(hb, 4)
    p2 = krylov.harmonic_ritz_general(hb, np.eye(j + 1, j), 4)
    assert p1.shape == p2.shape
    s1 = sla.orth(p1)
    s2 = sla.orth(p2)
    assert np.linalg.norm(s1 - s2 @ (s2.T @ s1)) < 1e-8


def test_harmonic_ritz_on_invariant_subspace_are_eigenvalues():
    g = np.random.default_rng(5)
    j = 6
    hm = np.triu(g.standard_normal((j, j)), -1) + 4 * np.eye(j)
    hb = np.vstack([hm, np.zeros((1, j))])
    theta = sla.eig(hb.T @ hb, hm.T, right=False)
    _same_spectrum(theta, np.linalg.eigvals(hm), 1e-9)


def test_select_ritz_pairs_and_cut():
    theta = np.array([0.1 + 0.2j, 0.1 - 0.2j, 0.05 + 0j, 3.0 + 0j, np.inf + 0j])
    vecs = np.eye(5, dtype=complex) + 1j * np.roll(np.eye(5), 1, axis=0)
    assert krylov.select_ritz(theta, vecs, 1).shape[1] == 1      # just 0.05
    assert krylov.select_ritz(theta, vecs, 2).shape[1] == 1      # pair does not fit
    assert krylov.select_ritz(theta, vecs, 3).shape[1] == 3      # 0.05 + pair
    assert krylov.select_ritz(theta, vecs, 5).shape[1] == 5      # inf last


def textbook_gmres(mat, z, m, tol, cap, u):
    """Independent restarted GMRES(m): MGS Arnoldi, lstsq, explicit restart
    from the implicit residual (d0 = 0)."""
    from oracle.fp import fl
    n = z.size
    d = np.zeros(n)
    r = z.copy()
    its = 0
    beta0 = np.linalg.norm(z)
    while np.linalg.norm(r) > tol * beta0 and its < cap:
        beta = np.linalg.norm(r)
        V = [fl(r / beta, u)]
        H = np.zeros((m + 1, m))
        for j in range(min(m, cap - its)):
            w = fl(mat @ V[j], u)
            basis = np.column_stack(V)
            h1 = basis.T @ w
            w = fl(w - basis @ h1, u)
            h2 = basis.T @ w
            w = fl(w - basis @ h2, u)
            H[: j + 1, j] = h1 + h2
            H[j + 1, j] = np.linalg.norm(w)
            V.append(fl(w / H[j + 1, j], u))
            c = np.zeros(j + 2)
            c[0] = beta
            y, *_ = np.linalg.lstsq(H[: j + 2, : j + 1], c, rcond=None)
            its += 1
            if np.linalg.norm(c - H[: j + 2, : j + 1] @ y) <= tol * beta0:
                break
        jj = len(V) - 1
        basis = np.column_stack(V)
        d = fl(d + basis[:, :jj] @ y, u)
        r = fl(r - basis @ (H[: jj + 1, :jj] @ y), u)
    return d, its


def test_k0_equals_textbook_restarted_gmres():
    g = np.random.default_rng(6)
    n = 120
    mat = np.eye(n) + 0.9 * g.standard_normal((n, n)) / np.sqrt(n)
    z = g.standard_normal(n)
    ap, a64 = _ops(mat, "fp64")
    d, rec = gcrodr(ap, a64, z, KrylovOptions(m=8, k=0, tau=1e-9, u="fp64", maxit=200), RecycleState())
    d_ref, its_ref = textbook_gmres(mat, z, 8, 1e-9, 200, "fp64")
    assert rec.its == its_ref
    assert np.linalg.norm(d - d_ref) <= 1e-8 * np.linalg.norm(d_ref)
    assert len(rec.cycles) > 1                 # restarts did happen


def test_recycle_pair_invariants_after_refresh():
    g = np.random.default_rng(7)
    n = 150
    ev = np.concatenate([np.geomspace(1e-3, 1e-1, 8), 1 + 0.1 * g.standard_normal(n - 8)])
    s = sla.qr(g.standard_normal((n, n)))[0]
    mat = s @ np.diag(ev) @ s.T
    ap, a64 = _ops(mat, "fp32")
    st = RecycleState()
    opts = KrylovOptions(m=20, k=5, tau=1e-4, u="fp32")
    d, rec = gcrodr(ap, a64, g.standard_normal(n), opts, st)
    assert st.U is not None and st.U.shape[1] in (4, 5)
    Cn = mat @ st.U                       # A U_k = C_k must be orthonormal
    assert np.linalg.norm(Cn.T @ Cn - np.eye(Cn.shape[1])) < 1e-4


def test_exact_deflation_one_iteration():
    g = np.random.default_rng(8)
    n, dsmall = 40, 6
    lam = np.array([0.05, 0.1, 0.2, 0.3, 0.45, 0.6])
    diag = np.ones(n)
    diag[-dsmall:] = lam
    mat = np.diag(diag)
    ap, a64 = _ops(mat, "fp64")
    z = g.standard_normal(n)
    opts_plain = KrylovOptions(m=20, k=0, tau=1e-10, u="fp64")
    _, rec_plain = gcrodr(ap, a64, z, opts_plain, RecycleState())
    assert rec_plain.its == dsmall + 1
    u0 = np.zeros((n, dsmall))
    u0[n - dsmall:, :] = g.standard_normal((dsmall, dsmall))   # spans e_lambda
    st = RecycleState(U=u0)
    opts_rec = KrylovOptions(m=20, k=dsmall, tau=1e-10, u="fp64")
    d, rec = gcrodr(ap, a64, z, opts_rec, st)
    assert rec.its == 1
    assert np.linalg.norm(mat @ d - z) <= 1e-9 * np.linalg.norm(z)


def test_recycled_second_system_needs_fewer_iterations():
    g = np.random.default_rng(9)
    n = 200
    ev = np.concatenate([np.geomspace(1e-4, 1e-2, 10), 1 + 0.3 * g.uniform(-1, 1, n - 10)])
    s = sla.qr(g.standard_normal((n, n)))[0]
    mat = s @ np.diag(ev) @ s.T
    ap, a64 = _ops(mat, "fp64")
    st = RecycleState()
    o = KrylovOptions(m=30, k=10, tau=1e-8, u="fp64")
    _, r1 = gcrodr(ap, a64, g.standard_normal(n), o, st)
    _, r2 = gcrodr(ap, a64, g.standard_normal(n), o, st)
    st0 = RecycleState()
    o0 = KrylovOptions(m=30, k=0, tau=1e-8, u="fp64")
    _, p2 = gcrodr(ap, a64, g.standard_normal(n), o0, st0)
    assert r2.its < p2.its


def test_mgs_is_the_sequential_recurrence_exactly():
    """Modified Gram-Schmidt (the oracle's ortho="mgs"): on dyadic inputs every
    fp64 operation is exact, so the oracle must reproduce the recurrence
    h_i = q_i . w_i, w_{i+1} = w_i - h_i q_i in exact rational arithmetic;
    on a non-orthogonal basis that differs from classical Gram-Schmidt, so a
    swap of the schemes is seen."""
    from fractions import Fraction
    from oracle.krylov import _orthogonalise
    g = np.random.default_rng(3)
    basis = g.integers(-2, 3, (6, 3)) / 4.0
    w = g.integers(-4, 5, 6) / 8.0
    wo, h = _orthogonalise(w.copy(), basis, "fp64", "mgs")
    wf = [Fraction(x) for x in w]
    hf = []
    for i in range(3):
        q = [Fraction(x) for x in basis[:, i]]
        hi = sum(a * b for a, b in zip(q, wf))
        hf.append(hi)
        wf = [a - hi * b for a, b in zip(wf, q)]
    assert [Fraction(x) for x in h] == hf
    assert [Fraction(x) for x in wo] == wf
    wc, hc = _orthogonalise(w.copy(), basis, "fp64", "cgs2")
    assert not np.array_equal(hc, h)


def test_mgs_arnoldi_relation_and_gmres_counts():
    """GMRES with modified Gram-Schmidt on the diagonal operator with d
    distinct eigenvalues: d iterations in fp64, as with CGS2."""
    from oracle.krylov import KrylovOptions, RecycleState, gcrodr
    d = 7
    lam = np.repeat(np.arange(1.0, d + 1.0), 5)
    n = lam.size
    z = np.random.default_rng(1).standard_normal(n)
    opts = KrylovOptions(m=20, k=0, tau=1e-12, maxit=0, u="fp64", ortho="mgs")
    dsol, rec = gcrodr(lambda v: lam * v, lambda y: lam[:, None] * y, z, opts, RecycleState())
    assert rec.its == d
    assert np.max(np.abs(lam * dsol - z)) <= 1e-10 * np.max(np.abs(z))
