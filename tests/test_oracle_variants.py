"""Pins for the speed variants of the oracle (uniform-precision products,
reuse of the recycled pair between refinement steps).

* reuse premise: at the end of a correction solve the recycled pair satisfies
  A-tilde U_k = C_k with orthonormal C_k, to the storage precision of the
  Krylov vectors, so it can stand in for QR(A-tilde U_k) when A is unchanged;
* reuse leaves the first refinement step (no recycled space yet) unchanged
  and the refinement still reaches its target;
* the uniform-precision product for u = fp64 equals M^-1 A v with M
  assembled from the factors (brute force), to kappa u;
* with uniform products the refinement at (fp32, fp64, double-double) still
  reaches the target on a system inside the uniform-precision bound.
"""
import numpy as np
import pytest

from oracle import Options, factor, refine, solve
from oracle.krylov import RecycleState
from synthetic import randsvd_problem

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def test_recycled_pair_invariant_holds_after_a_solve():
    p = randsvd_problem(150, 1e5, 2)
    o = Options(uf="fp16", u="fp32", ur="fp64", m=12, k=4, tau=1e-4, nb=64, keep_recycle=True)
    f = factor(p.a, o)
    st = RecycleState()
    x, info = solve(f, p.b, st)
    assert info.status == refine.STATUS_OK
    assert st.C is not None and st.U is not None
    au = refine.atilde64(f, st.U)
    rel = np.linalg.norm(au - st.C) / np.linalg.norm(st.C)
    orth = np.linalg.norm(st.C.T @ st.C - np.eye(st.C.shape[1]))
    # both to the storage precision of the Krylov vectors (fp32)
    assert rel <= 100 * U32
    assert orth <= 100 * U32


@pytest.mark.parametrize("k", [4, 8])
def test_reuse_keeps_first_step_and_converges(k):
    p = randsvd_problem(200, 1e5, 4)
    base = dict(uf="fp16", u="fp32", ur="fp64", m=16, k=k, tau=1e-4, nb=64)
    f0 = factor(p.a, Options(**base))
    _, info0 = solve(f0, p.b)
    f1 = factor(p.a, Options(**base, reuse_recycle=True))
    _, info1 = solve(f1, p.b)
    assert info1.its[0] == info0.its[0]
    assert info1.status == refine.STATUS_OK
    assert info1.berr[-1] <= 1e-14


def test_uniform_product_equals_assembled_m():
    g = np.random.default_rng(7)
    a = g.standard_normal((40, 40))
    f = factor(a, Options(uf="fp32", u="fp64", ur="dd", matvec="u", tau=1e-8, nb=16))
    lu = f.L @ f.U
    mm = np.empty_like(lu)
    mm[f.perm] = lu
    mm = np.ldexp(mm, -f.e)
    v = g.standard_normal(40)
    ref = np.linalg.solve(mm, a @ v)
    got = refine.atilde_uniform(f, v)
    kappa = np.linalg.cond(mm)
    assert np.max(np.abs(got - ref)) <= 10 * kappa * 40 * U64 * np.max(np.abs(ref))


def test_uniform_refinement_converges():
    p = randsvd_problem(200, 1e8, 4)
    o = Options(uf="fp32", u="fp64", ur="dd", m=20, k=5, tau=1e-8, nb=64, matvec="u")
    f = factor(p.a, o)
    x, info = solve(f, p.b)
    assert info.status == refine.STATUS_OK
    assert info.berr[-1] <= 1e-14


def test_uniform_rejected_for_fp32_working_precision():
    with pytest.raises(ValueError):
        Options(uf="fp16", u="fp32", ur="fp64", matvec="u").validate()


def test_batch_specs_follow_the_stated_distribution():
    """The uneven batch's specifications: sizes, conditioning and right-hand
    side counts inside their ranges, reproducible from the seed, and spread
    over the ranges (512 draws)."""
    from synthetic import batch_specs
    sp = batch_specs(512, 1)
    assert sp == batch_specs(512, 1)
    ns = np.array([d["n"] for d in sp])
    ks = np.log10([d["kappa"] for d in sp])
    rs = np.array([d["nrhs"] for d in sp])
    assert ns.min() >= 128 and ns.max() <= 2048 and ks.min() >= 1 and ks.max() <= 8
    assert rs.min() >= 1 and rs.max() <= 8 and set(rs) == set(range(1, 9))
    assert abs(np.mean(ns) - 1088) < 60 and abs(np.mean(ks) - 4.5) < 0.25
    assert len({d["seed"] for d in sp}) == 512
