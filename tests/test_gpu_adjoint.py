"""GPU parity of the adjoint path: A^T lambda = g with the transposed
factors (gmresir_solve_transposed), its preconditioned products, and the
gradient of L = 0.5 ||x - y||^2 through x = A^-1 b (the autograd Function).

Bars: products with shared factors within the LU-solve backward error
bound (M^-T v) and a first-order forward bound (M^-T A_u^T v);
solves: identical refinement-step counts, Arnoldi iterations within +-2
(identical with shared factors), backward error <= 8 n u, forward error
within 10x the oracle's; gradients: central finite differences of the fp64
loss at n = 64 and the dense fp64 gradient at n = 1024.
"""
import numpy as np
import pytest

from gpu_util import U64, encode_factors, lib_options, log, oracle_options
from oracle import refine
from synthetic import randsvd_problem

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


def _import(lib, p, f, o):
    return lib.import_factors(_dev(p.a), _dev(encode_factors(f.lu, o.uf).view(np.int16)),
                              f.ipiv.astype(np.int32), f.e, **lib_options(o))


def _lu_t_backward_error(f, rhs, z):
    """max |rhs - M^T z| / max(|M|^T |z|) with M^T = 2^-e U^T L^T P, the
    residual in extended precision (transposed LU-solve backward error)."""
    ld = np.longdouble
    zp = z[f.perm]
    mz = f.U.T.astype(ld) @ (f.L.T.astype(ld) @ zp.astype(ld))
    r = (np.asarray(rhs, dtype=ld) - np.ldexp(mz, -f.e)).astype(np.float64)
    den = np.ldexp(np.abs(f.U).T @ (np.abs(f.L).T @ np.abs(zp)), -f.e)
    return np.max(np.abs(r)) / np.max(den)


@pytest.mark.parametrize("n", [100, 333, 1024])
def test_transposed_products_with_shared_factors(lib, n):
    """M^-T v within the transposed LU-solve backward error bound 3 n u^2;
    M^-T A_u^T v within its first-order forward bound from the summation
    order of the product with A_u^T."""
    p = randsvd_problem(n, 1e5, 7)
    o = oracle_options()
    f = refine.factor(p.a, o)
    log(f"[apply-t] n={n}")
    h = _import(lib, p, f, o)
    g = np.random.default_rng(n + 5)
    v = g.standard_normal(n).astype(np.float32).astype(np.float64)
    y2 = h.apply(2, _dev(v)).cpu().numpy()
    y3 = h.apply(3, _dev(v)).cpu().numpy()
    h.free()
    r2 = refine.minv_t(f, v)
    r3 = refine.minv_t(f, f.au.T @ v)
    e2 = np.linalg.norm(y2 - r2) / np.linalg.norm(r2)
    e3 = np.linalg.norm(y3 - r3) / np.linalg.norm(r3)
    b2 = _lu_t_backward_error(f, v, y2)
    # the products with A_u^T differ in summation order only: bounded by
    # n u |M^-T| (|A_u|^T |v|), relative to the result
    mt = np.abs(refine.minv_t(f, np.eye(n)))
    b3 = n * U64 * np.linalg.norm(mt @ (np.abs(f.au).T @ np.abs(v))) / np.linalg.norm(r3)
    log(f"[apply-t] n={n} rel diff M^-T v {e2:.2e} (backward error / u^2 {b2 / U64:.2f})  "
        f"M^-T A_u^T v {e3:.2e} (bound {b3:.2e})")
    assert b2 <= 3 * n * U64 and e3 <= b3


def _check(p, g, lam, info, lam_ref, info_ref, n, shared):
    log(f"  oracle: status={info_ref.status} steps={info_ref.steps} its={info_ref.its} "
        f"berr={info_ref.berr[-1]:.2e}")
    log(f"  gpu:    status={info['status']} steps={info['steps']} its={info['its']} "
        f"berr={info['berr'][-1]:.2e}")
    assert info["status"] == info_ref.status
    assert info["steps"] == info_ref.steps
    if shared:
        assert info["its"] == info_ref.its
    for a, b in zip(info["its"], info_ref.its):
        assert abs(a - b) <= 2
    assert info["berr"][-1] <= 8 * n * U64
    # backward error recomputed here in fp64
    r = g - p.a.T @ lam
    eta = np.max(np.abs(r)) / (np.max(np.sum(np.abs(p.a), axis=0)) * np.max(np.abs(lam))
                               + np.max(np.abs(g)))
    assert eta <= 8 * n * U64
    exact = np.linalg.solve(p.a.T, g)
    fe = np.max(np.abs(lam - exact)) / np.max(np.abs(exact))
    fo = np.max(np.abs(lam_ref - exact)) / np.max(np.abs(exact))
    log(f"  ferr gpu {fe:.2e} oracle {fo:.2e}")
    assert fe <= 10 * fo + 10 * n * U64


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("k", [5, 0])
def test_solve_transposed_shared_factors(lib, seed, k):
    p = randsvd_problem(100, 1e4, seed)
    o = oracle_options(m=20, k=k)
    f = refine.factor(p.a, o)
    g = np.random.default_rng(seed + 100).standard_normal(100)
    lam_ref, info_ref = refine.solve_transposed(f, g)
    log(f"[solve-t-shared] seed={seed} k={k}")
    h = _import(lib, p, f, o)
    lam, info = h.solve_transposed(_dev(g))
    h.free()
    _check(p, g, lam.cpu().numpy(), info, lam_ref, info_ref, 100, True)


# seeds chosen so that the oracle's backward errors clear the 1e-14 target by
# more than a decade at every step (the step count is not decided by rounding)
@pytest.mark.parametrize("n,kappa,k,seed", [(513, 1e4, 10, 2), (1100, 1e4, 10, 1),
                                            (900, 1e4, 10, 3), (300, 1e4, 0, 2)])
def test_solve_transposed_full_path(lib, n, kappa, k, seed):
    p = randsvd_problem(n, kappa, seed)
    o = oracle_options(m=30, k=k)
    f = refine.factor(p.a, o)
    g = np.random.default_rng(n).standard_normal(n)
    lam_ref, info_ref = refine.solve_transposed(f, g)
    log(f"[solve-t] n={n} kappa={kappa:g} k={k}")
    h = lib.factor(_dev(p.a), **lib_options(o))
    # the forward solve first: the adjoint keeps a recycle space of its own
    x, xinfo = h.solve(_dev(p.b))
    assert xinfo["status"] == 0
    lam, info = h.solve_transposed(_dev(g))
    h.free()
    _check(p, g, lam.cpu().numpy(), info, lam_ref, info_ref, n, False)


def _loss_np(a, b, y):
    x = np.linalg.solve(a, b)
    return 0.5 * float(np.sum((x - y) ** 2))


def _grads(lib, a, b, y, **opts):
    from paper_2201_09827_amd import autograd as ga
    at = _dev(a).requires_grad_(True)
    bt = _dev(b).requires_grad_(True)
    x = ga.solve(at, bt, **opts)
    loss = 0.5 * torch.sum((x - _dev(y)) ** 2)
    loss.backward()
    return at.grad.cpu().numpy(), bt.grad.cpu().numpy(), x.detach().cpu().numpy()


def test_gradient_finite_differences_n64(lib):
    n = 64
    p = randsvd_problem(n, 1e3, 4)
    rng = np.random.default_rng(21)
    y = rng.standard_normal(n)
    log("[grad] n=64 central differences")
    da, db, _ = _grads(lib, p.a, p.b, y, m=10, k=3)
    h = 1e-8
    for _ in range(4):
        e_a = rng.standard_normal((n, n))
        e_b = rng.standard_normal(n)
        fd = (_loss_np(p.a + h * e_a, p.b + h * e_b, y)
              - _loss_np(p.a - h * e_a, p.b - h * e_b, y)) / (2 * h)
        an = float(np.sum(da * e_a) + db @ e_b)
        log(f"[grad] fd {fd:.10e} adjoint {an:.10e}")
        assert abs(fd - an) <= 1e-5 * abs(an)


def test_gradient_dense_reference_n1024(lib):
    n = 1024
    p = randsvd_problem(n, 1e4, 6)
    y = np.random.default_rng(5).standard_normal(n)
    log("[grad] n=1024 dense fp64 reference")
    da, db, x = _grads(lib, p.a, p.b, y, m=30, k=10)
    xr = np.linalg.solve(p.a, p.b)
    lr = np.linalg.solve(p.a.T, xr - y)
    ref_a = -np.outer(lr, xr)
    ea = np.max(np.abs(da - ref_a)) / np.max(np.abs(ref_a))
    eb = np.max(np.abs(db - lr)) / np.max(np.abs(lr))
    kappa = np.linalg.cond(p.a, np.inf)
    log(f"[grad] n=1024 rel err dA {ea:.2e} db {eb:.2e} (kappa_inf {kappa:.1e})")
    assert ea <= 10 * kappa * n * U64 and eb <= 10 * kappa * n * U64


# moderately conditioned systems: at kappa ~ 1e5 the counts of a sweep
# change by tens of steps with the summation order of the CPU's own BLAS
@pytest.mark.parametrize("n,kappa,seed,m,kmax", [(100, 1e4, 3, 20, 8), (300, 1e4, 4, 10, 6),
                                                 (256, 1e4, 1, 8, 6)])
def test_choose_k_shared_factors(lib, n, kappa, seed, m, kmax):
    """Automatic k on the oracle's factors: the iteration count of every k
    within +-2 of the oracle's, the same limit, and a chosen k whose count is
    within 2 of the oracle's minimum (the same k when the oracle's minimum is
    unique by more than 4 steps)."""
    p = randsvd_problem(n, kappa, seed)
    o = oracle_options(m=m, k=kmax)
    f = refine.factor(p.a, o)
    kb_ref, its_ref = refine.choose_k(f, p.b, kmax)
    log(f"[choose-k] n={n} oracle k={kb_ref} its={its_ref}")
    h = _import(lib, p, f, o)
    kb, its, status = h.choose_k(_dev(p.b), kmax)
    h.free()
    log(f"[choose-k] n={n} gpu    k={kb} its={its} status={status}")
    assert status == 0
    for a, b in zip(its, its_ref):
        assert (a < 0) == (b < 0)
        assert a < 0 or abs(a - b) <= 2
    best = min(t for t in its_ref if t >= 0)
    assert its[kb] == min(t for t in its if t >= 0)
    assert its_ref[kb] >= 0 and its_ref[kb] - best <= 2
    others = [t for k, t in enumerate(its_ref) if t >= 0 and k != kb_ref]
    if not others or min(others) > best + 4:
        assert kb == kb_ref
