"""GPU parity: the HIP library against the CPU oracle on the same seeded
inputs (all calls go through the C ABI via the ctypes binding).

Bars:
* LU: pivots identical; u_f entries identical except rare one-ulp splits of
  the fp32-accumulated trailing update; componentwise backward error within
  the blocked-GEPP bound.
* preconditioned products with identical factors: fp64 results within the
  LU-solve backward error bound; rounded to u, nearly all entries identical.
* end-to-end: identical refinement-step counts, GMRES iterations within +-2
  per step, normwise backward error <= 8 n u, forward error within 10x the
  oracle's.
"""
import numpy as np
import pytest

from gpu_util import (NB, U64, decode_factors, encode_factors, lib_options, log,
                      oracle_factors, oracle_options, ulp_distance)
from oracle import fp, refine
from oracle.lu import unpack
from synthetic import prolate_problem, randsvd_problem

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2201_09827_amd as g
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g.load_library()
    return g


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("n,uf", [(100, "fp16"), (257, "fp16"), (1000, "fp16"),
                                  (300, "bf16"), (200, "fp32"), (1000, "fp32")])
def test_lu_factors_match_oracle(lib, n, uf):
    p = randsvd_problem(n, 1e4, 11)
    log(f"[lu] n={n} uf={uf}")
    h = lib.factor(_dev(p.a), uf=uf, m=20, k=5)
    assert h.status == 0
    raw, ipiv, e = h.export_factors()
    h.free()
    res, e_ref, af = oracle_factors(p.a, uf)
    assert e == e_ref
    lu_gpu = decode_factors(raw, uf)
    nbk = min(NB, n)
    # the first block column is factored with the same fp32 fused
    # multiply-add sequence on both sides: identical pivots and entries, and
    # the block row right of it (fp32 solve with the stored triangle) too
    assert np.array_equal(ipiv[:nbk], res.ipiv[:nbk])
    perm = np.arange(n)
    for i, j in enumerate(ipiv):
        perm[[i, j]] = perm[[j, i]]
    # rows of the first block column, matched by original row (later
    # interchanges only move them), and the first block row
    inv_g = np.argsort(perm)
    inv_o = np.argsort(res.perm)
    d_col = ulp_distance(lu_gpu[inv_g, :nbk], res.lu[inv_o, :nbk], uf)
    d_row = ulp_distance(lu_gpu[:nbk, nbk:], res.lu[:nbk, nbk:], uf)
    d = ulp_distance(lu_gpu, res.lu, uf)
    diverge = int(np.argmax(ipiv != res.ipiv)) if np.any(ipiv != res.ipiv) else n
    log(f"[lu] n={n} uf={uf} first block column/row max ulp {d_col.max():.1f}/"
        f"{d_row.max() if d_row.size else 0:.1f}; pivots identical up to column {diverge}; "
        f"entries > 1 ulp apart {np.mean(d > 1):.2e}")
    if d_row.size and d_row.max() > 0:
        bad = np.argwhere(d_row > 0)[:8]
        log(f"[lu] first block row mismatches (row, col): {bad.tolist()} "
            f"gpu {[lu_gpu[r, nbk + c] for r, c in bad]} oracle {[res.lu[r, nbk + c] for r, c in bad]}")
    assert d_col.max() == 0.0
    assert d_row.size == 0 or d_row.max() == 0.0
    if uf == "fp32":
        # fp32 factors: the trailing update is accumulated in fp64 on both
        # sides and rounded once, so the factors agree everywhere but for
        # fp64 summation-order ties
        assert np.array_equal(ipiv, res.ipiv)
        assert np.mean(d > 0) <= 1e-4
    # later block columns see the fp32-accumulated trailing update (the CPU
    # reference accumulates exactly), so near-ties may pick other pivots:
    # the GPU factors must still satisfy the blocked-GEPP backward error bound
    L, U = unpack(lu_gpu)
    lhs = np.abs(af[perm] - L @ U)
    rhs = np.abs(L) @ np.abs(U)
    c = 2 * (n // NB + 3) * fp.unit_roundoff(uf)
    assert np.all(lhs <= c * rhs + 1e-300)
    assert np.all(np.abs(np.tril(L, -1)) <= 1.0)      # partial pivoting


def _lu_backward_error(f, rhs, z, extra=None):
    """max |rhs - M z| / max(|M| |z| (+ extra)) with M = 2^-e P^T L U, the
    residual in extended precision (LU-solve backward error, normwise)."""
    ld = np.longdouble
    zs = np.ldexp(z, -f.e)
    lu = f.L.astype(ld) @ (f.U.astype(ld) @ zs.astype(ld))
    mz = np.empty_like(lu)
    mz[f.perm] = lu
    r = (np.asarray(rhs, dtype=ld) - mz).astype(np.float64)
    a = np.abs(f.L) @ (np.abs(f.U) @ np.abs(zs))
    den = np.empty_like(a)
    den[f.perm] = a
    if extra is not None:
        den = den + extra
    return np.max(np.abs(r)) / np.max(den)


@pytest.mark.parametrize("n", [100, 333, 1024])
def test_preconditioned_products_with_shared_factors(lib, n):
    """M^-1 v and A-tilde v with the oracle's factors, in fp64 (precision u^2):
    each within the backward error bound of a solve with the LU factors,
    |r| <= 3 n u^2 (|L||U||z| (+ |A_u||v|)); the forward difference from the
    oracle's substitution is rounding-order noise amplified by the condition
    of U, logged; once rounded to u nearly every entry is identical."""
    p = randsvd_problem(n, 1e5, 5)
    o = oracle_options()
    f = refine.factor(p.a, o)
    log(f"[apply] n={n}")
    h = lib.import_factors(_dev(p.a), _dev(encode_factors(f.lu, "fp16").view(np.int16)),
                           f.ipiv.astype(np.int32), f.e, **lib_options(o))
    g = np.random.default_rng(n)
    v = fp.fl32(g.standard_normal(n))
    y0 = h.apply(0, _dev(v)).cpu().numpy()
    y1 = h.apply(1, _dev(v)).cpu().numpy()
    h.free()
    r0 = refine.minv_hi(f, v, "fp64")
    r1 = refine.minv_hi(f, f.au @ v, "fp64")
    e0 = np.linalg.norm(y0 - r0) / np.linalg.norm(r0)
    e1 = np.linalg.norm(y1 - r1) / np.linalg.norm(r1)
    # A_u v exactly (fp32 products are exact in fp64; the sum in extended precision)
    w = f.au.astype(np.longdouble) @ v.astype(np.longdouble)
    b0 = _lu_backward_error(f, v, y0)
    b1 = _lu_backward_error(f, w, y1, extra=np.abs(f.au) @ np.abs(v))
    log(f"[apply] n={n} rel diff from oracle M^-1 v {e0:.2e}  A~v {e1:.2e}; "
        f"backward error / u^2 {b0 / U64:.2f} {b1 / U64:.2f}")
    assert b0 <= 3 * n * U64 and b1 <= 3 * n * U64
    # once rounded to u (fp32) nearly every entry is identical
    same = np.mean(fp.fl32(y1) == fp.fl32(r1))
    assert same > 0.99


@pytest.mark.parametrize("n,uf,u", [(4097, "fp16", "fp32"), (8192, "fp16", "fp32"),
                                    (8192, "bf16", "fp32"), (16384, "fp16", "fp32"),
                                    (16384, "fp32", "fp64")])
def test_preconditioner_full_size_properties(lib, n, uf, u):
    """At the full sizes (oracle too slow): y = M^-1 v must satisfy
    L U (2^-e y) = P v to the fp64 substitution bound with the library's own
    factors (checked on the GPU in fp64), likewise A-tilde v against P A_u v;
    the same launch configuration as the solves (u = fp64: the double-double
    kernels, A_u = A)."""
    from synthetic import randsvd_problem_torch
    log(f"[apply-full] n={n} uf={uf} u={u}")
    a, _, _ = randsvd_problem_torch(n, 1e2, 3, "cuda")
    ur = "dd" if u == "fp64" else "fp64"
    h = lib.factor(a, uf=uf, u=u, ur=ur, m=30, k=10)
    assert h.status == 0
    raw, ipiv, e = h.export_factors()
    if uf == "fp16":
        lu = torch.from_numpy(raw.view(np.float16)).to("cuda").to(torch.float64)
    elif uf == "bf16":
        lu = torch.from_numpy(raw.view(np.int16)).to("cuda").view(torch.bfloat16).to(torch.float64)
    else:
        lu = torch.from_numpy(raw).to("cuda").to(torch.float64)
    del raw
    L = torch.tril(lu, -1) + torch.eye(n, dtype=torch.float64, device="cuda")
    U = torch.triu(lu)
    del lu
    perm = np.arange(n)
    for i, j in enumerate(ipiv):
        perm[[i, j]] = perm[[j, i]]
    pt = torch.from_numpy(perm).to("cuda")
    # the library's own factors at this size: partial pivoting (|L| <= 1) and
    # the blocked-GEPP componentwise backward error of P A_f = L U, in fp64
    af = a * 2.0 ** e
    af = {"fp16": af.half(), "bf16": af.bfloat16()}.get(uf, af.float()).double()
    lmax = torch.max(torch.abs(torch.tril(L, -1))).item()
    lhs = torch.abs(af[pt] - L @ U)
    rhs = torch.abs(L) @ torch.abs(U)
    c = 2 * (n // NB + 3) * fp.unit_roundoff(uf)
    worst = torch.max(lhs / (c * rhs + 1e-300)).item()
    log(f"[apply-full] n={n} max|L| {lmax:.3f}; backward error of P A_f = L U / bound {worst:.3f}")
    assert lmax <= 1.0
    assert worst <= 1.0
    del af, lhs, rhs
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    v = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
    if u == "fp32":
        v = v.float().double()
    au = a.float().double() if u == "fp32" else a
    for op, rhs in ((0, v[pt]), (1, (au @ v)[pt])):
        y = h.apply(op, v) * 2.0 ** (-e)
        lhs = L @ (U @ y)
        res = torch.max(torch.abs(lhs - rhs)).item()
        bound = (torch.max(torch.sum(torch.abs(L), 1)) * torch.max(torch.sum(torch.abs(U), 1))
                 * torch.max(torch.abs(y))).item()
        rel = res / bound
        log(f"[apply-full] n={n} op={op} relative residual {rel:.2e}")
        assert rel <= 4 * n * U64
    h.free()


def _run_oracle(p, o, f=None):
    f = refine.factor(p.a, o) if f is None else f
    x, info = refine.solve(f, p.b)
    return x, info, f


def _ferr(x, xt):
    return float(np.max(np.abs(x - xt)) / np.max(np.abs(xt)))


def _compare(p, x_ref, info_ref, x, info, n):
    log(f"  oracle: status={info_ref.status} steps={info_ref.steps} its={info_ref.its} "
        f"berr={info_ref.berr[-1]:.2e}")
    log(f"  gpu:    status={info['status']} steps={info['steps']} its={info['its']} "
        f"berr={info['berr'][-1]:.2e} t_solve={info['t_solve_s'] * 1e3:.2f} ms")
    assert info["status"] == info_ref.status
    assert info["steps"] == info_ref.steps
    for a, b in zip(info["its"], info_ref.its):
        assert abs(a - b) <= 2
    assert info["berr"][-1] <= 8 * n * U64
    if p.x_true is not None:
        fe, fo = _ferr(x, p.x_true), _ferr(x_ref, p.x_true)
        log(f"  ferr gpu {fe:.2e} oracle {fo:.2e}")
        assert fe <= 10 * fo + 10 * n * U64


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("k", [5, 0])
def test_solve_shared_factors_config_small(lib, seed, k):
    p = randsvd_problem(100, 1e4, seed)
    o = oracle_options(m=20, k=k)
    x_ref, info_ref, f = _run_oracle(p, o)
    log(f"[solve-shared] seed={seed} k={k}")
    h = lib.import_factors(_dev(p.a), _dev(encode_factors(f.lu, "fp16").view(np.int16)),
                           f.ipiv.astype(np.int32), f.e, **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    _compare(p, x_ref, info_ref, x.cpu().numpy(), info, 100)
    assert info["its"] == info_ref.its


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("k", [5, 0])
def test_solve_full_path_config_small(lib, seed, k):
    p = randsvd_problem(100, 1e4, seed)
    o = oracle_options(m=20, k=k)
    x_ref, info_ref, _ = _run_oracle(p, o)
    log(f"[solve-full] n=100 seed={seed} k={k}")
    h = lib.factor(_dev(p.a), **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    _compare(p, x_ref, info_ref, x.cpu().numpy(), info, 100)


@pytest.mark.parametrize("n,kappa,m,k", [(513, 1e4, 30, 10), (1100, 1e3, 30, 10),
                                         (777, 1e4, 40, 8)])
def test_solve_full_path_ragged_sizes(lib, n, kappa, m, k):
    # seed 2: the oracle's backward errors clear 1e-14 by > 1.7 decades at
    # every step, so the step count is not decided by rounding noise
    p = randsvd_problem(n, kappa, 2)
    o = oracle_options(m=m, k=k)
    x_ref, info_ref, _ = _run_oracle(p, o)
    log(f"[solve-full] n={n} kappa={kappa:g} m={m} k={k}")
    h = lib.factor(_dev(p.a), **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    _compare(p, x_ref, info_ref, x.cpu().numpy(), info, n)


@pytest.mark.parametrize("uf,kind", [("bf16", "prolate"), ("fp32", "prolate"),
                                     ("bf16", "randsvd")])
def test_solve_other_factor_precisions(lib, uf, kind):
    if kind == "prolate":
        p = prolate_problem(300, 0.495, seed=3)     # kappa_2 ~ 9e2
    else:
        p = randsvd_problem(300, 1e3, 3)
    o = oracle_options(uf=uf, m=20, k=5)
    x_ref, info_ref, _ = _run_oracle(p, o)
    log(f"[solve-full] {kind} n=300 uf={uf}")
    h = lib.factor(_dev(p.a), **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    _compare(p, x_ref, info_ref, x.cpu().numpy(), info, 300)


@pytest.mark.parametrize("n", [64, 200, 333])
def test_double_double_products_with_shared_factors(lib, n):
    """u = fp64: M^-1 v and A-tilde v in double-double with the oracle's fp32
    factors; after rounding to fp64 the two agree to an ulp or so (the sums
    differ only in order, far below fp64 resolution)."""
    p = randsvd_problem(n, 1e8, 6)
    o = oracle_options(uf="fp32", u="fp64", ur="dd", tau=1e-8)
    f = refine.factor(p.a, o)
    log(f"[apply-dd] n={n}")
    h = lib.import_factors(_dev(p.a), _dev(encode_factors(f.lu, "fp32")),
                           f.ipiv.astype(np.int32), f.e, **lib_options(o))
    g = np.random.default_rng(n + 11)
    v = g.standard_normal(n)
    y0 = h.apply(0, _dev(v)).cpu().numpy()
    y1 = h.apply(1, _dev(v)).cpu().numpy()
    h.free()
    r0 = refine.minv_hi(f, v, "dd")
    r1 = refine.atilde(f, v)
    for name, y, r in (("M^-1 v", y0, r0), ("A~v", y1, r1)):
        err = np.max(np.abs(y - r)) / np.max(np.abs(r))
        same = np.mean(y == r)
        log(f"[apply-dd] n={n} {name}: max rel diff {err:.2e}, identical {same:.3f}")
        assert err <= 4 * U64
        assert same > 0.9
    # the fp64 solve of the same system is visibly less accurate
    r64 = refine.minv_hi(f, v, "fp64")
    log(f"[apply-dd] n={n} fp64 solve differs by "
        f"{np.max(np.abs(r64 - r0)) / np.max(np.abs(r0)):.2e}")


def test_solve_fp64_shared_factors(lib):
    """u = fp64 with the oracle's own fp32 factors: a system near the edge of
    convergence (kappa u_f ~ 60, three GCRO-DR cycles, 49 Arnoldi steps)
    isolates the fp64 Arnoldi and double-double paths from the LU."""
    p = randsvd_problem(200, 1e9, 4)
    o = oracle_options(uf="fp32", u="fp64", ur="dd", m=20, k=5, tau=1e-8)
    x_ref, info_ref, f = _run_oracle(p, o)
    log("[solve-dd-shared] randsvd n=200 kappa=1e9")
    h = lib.import_factors(_dev(p.a), _dev(encode_factors(f.lu, "fp32")),
                           f.ipiv.astype(np.int32), f.e, **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    _compare(p, x_ref, info_ref, x.cpu().numpy(), info, 200)


@pytest.mark.parametrize("kind,n,m,k,kappa,seed", [("randsvd", 300, 5, 2, 1e8, 3),
                                                    ("randsvd", 200, 4, 2, 1e8, 4),
                                                    ("randsvd", 333, 20, 0, 1e8, 4),
                                                    ("prolate", 240, 6, 3, 0.0, 3)])
def test_solve_fp64_working_precision(lib, kind, n, m, k, kappa, seed):
    """(u_f, u, u_r) = (fp32, fp64, double-double) end to end, tau = 1e-8
    (randsvd: 11-12 Arnoldi steps over four GCRO-DR cycles; prolate
    w = 0.48: two refinement steps, the second with the recycled space)."""
    if kind == "prolate":
        p = prolate_problem(n, 0.48, seed=seed)
    else:
        p = randsvd_problem(n, kappa, seed)
    o = oracle_options(uf="fp32", u="fp64", ur="dd", m=m, k=k, tau=1e-8)
    x_ref, info_ref, _ = _run_oracle(p, o)
    log(f"[solve-dd] {kind} n={n} m={m} k={k}")
    h = lib.factor(_dev(p.a), **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    _compare(p, x_ref, info_ref, x.cpu().numpy(), info, n)


def test_edge_cases(lib):
    log("[edge] identity, n=1, zero column, NaN, imax")
    n = 70
    b = np.linspace(-1, 1, n)
    h = lib.factor(_dev(np.eye(n)), m=5, k=2)
    x, info = h.solve(_dev(b))
    h.free()
    assert info["status"] == 0 and info["steps"] == 0
    assert np.array_equal(x.cpu().numpy(), b)
    h = lib.factor(_dev(np.array([[4.0]])), m=1, k=0)
    x, info = h.solve(_dev(np.array([2.0])))
    h.free()
    assert info["status"] == 0 and abs(x.item() - 0.5) < 1e-15
    a = np.random.default_rng(0).standard_normal((90, 90))
    a[:, 37] = 0.0
    h = lib.factor(_dev(a), m=10, k=2)
    assert h.status == 1
    x, info = h.solve(_dev(np.ones(90)))
    assert info["status"] == 1 and info["singular_col"] == 38
    h.free()
    a = np.random.default_rng(1).standard_normal((40, 40))
    a[3, 4] = np.nan
    h = lib.factor(_dev(a), m=10, k=2)
    assert h.status == 2
    h.free()
    p = randsvd_problem(100, 1e4, 1)
    h = lib.factor(_dev(p.a), m=20, k=5)
    bb = p.b.copy()
    bb[5] = np.inf
    _, info = h.solve(_dev(bb))
    assert info["status"] == 2
    h.free()
    h = lib.factor(_dev(p.a), m=20, k=5, imax=1)
    x, info = h.solve(_dev(p.b))
    h.free()
    o = oracle_options(m=20, k=5, imax=1)
    _, info_ref, _ = _run_oracle(p, o)
    assert info["status"] == 3 == info_ref.status
    assert info["steps"] == 1 and np.all(np.isfinite(x.cpu().numpy()))
    with pytest.raises(lib.GmresirError):
        lib.factor(_dev(p.a), m=5, k=5)


def test_keep_recycle_across_right_hand_sides(lib):
    """The recycled space carried between right-hand sides (the algorithm's
    last line) follows the oracle; shared factors isolate the solve phase."""
    from oracle.krylov import RecycleState
    p = randsvd_problem(513, 1e4, 2)
    g = np.random.default_rng(9)
    o = oracle_options(m=30, k=8)
    o.keep_recycle = True
    f = refine.factor(p.a, o)
    st = RecycleState()
    log("[keep-recycle] n=513 three right-hand sides, shared factors")
    h = lib.import_factors(_dev(p.a), _dev(encode_factors(f.lu, "fp16").view(np.int16)),
                           f.ipiv.astype(np.int32), f.e, keep_recycle=1, **lib_options(o))
    for j in range(3):
        b = p.a @ g.uniform(-1, 1, 513)
        x_ref, info_ref = refine.solve(f, b, st)
        x, info = h.solve(_dev(b))
        log(f"  rhs {j}: oracle {info_ref.its} {['%.1e' % e for e in info_ref.berr]} "
            f"gpu {info['its']} {['%.1e' % e for e in info['berr']]}")
        assert info["steps"] == info_ref.steps
        for a_, b_ in zip(info["its"], info_ref.its):
            assert abs(a_ - b_) <= 2
        assert info["recycle_dim"] == st.dim
    h.free()


def test_solve_largest_recycle_dimensions_shared_factors(lib):
    """m = 95, k = 42 (the largest m with (m + 1) k <= 4096): the small
    products of the recycle space then have (k + m + 1) k = 5796 outputs."""
    # first correction 179 Arnoldi steps (full cycles of 95 with the recycle
    # refresh); counts identical with 1 and 8 BLAS threads in the oracle
    p = randsvd_problem(300, 1e6, 1)
    o = oracle_options(m=95, k=42)
    x_ref, info_ref, f = _run_oracle(p, o)
    log("[solve-shared] n=300 m=95 k=42")
    h = lib.import_factors(_dev(p.a), _dev(encode_factors(f.lu, "fp16").view(np.int16)),
                           f.ipiv.astype(np.int32), f.e, **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    _compare(p, x_ref, info_ref, x.cpu().numpy(), info, 300)


def test_kernel_timing_records_and_sampling(lib):
    """Launch timing (opts.timing): every launch of a timed class, or every
    s-th with bits 8-15; 16 block columns at n = 1024."""
    p = randsvd_problem(1024, 1e2, 1)
    a, b = _dev(p.a), _dev(p.b)
    full = lib.factor(a, timing=1)
    x1, _ = full.solve(b)
    s1 = {r["name"]: r for r in full.kernel_stats()}
    full.free()
    samp = lib.factor(a, timing=1 | (8 << 8))
    x2, _ = samp.solve(b)
    s2 = {r["name"]: r for r in samp.kernel_stats()}
    samp.free()
    log(f"[timing] every launch {s1['lu_panel']['launches']}, every 8th {s2['lu_panel']['launches']}")
    assert s1["lu_panel"]["launches"] == 16 and s2["lu_panel"]["launches"] == 2
    assert s1["lu_panel"]["total_ms"] > 0 and s2["lu_panel"]["total_ms"] > 0
    assert torch.equal(x1, x2)
    with pytest.raises(lib.GmresirError):
        lib.factor(a, timing=1 << 24)
