"""GPU parity of the speed variants: uniform-precision products for u = fp64
(SGMRES-IR / RSGMRES-IR, opts.matvec_u) and reuse of the recycled pair
between refinement steps (opts.reuse_recycle).  Bars as for the main path:
identical refinement-step counts, Arnoldi iterations identical with the
oracle's own factors and within +-2 otherwise, backward error <= 8 n u,
forward error within 10x the oracle's."""
import numpy as np
import pytest

from gpu_util import U64, encode_factors, lib_options, log, oracle_options
from oracle import refine
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


def _compare(p, x_ref, info_ref, x, info, n, shared):
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
    fe = np.max(np.abs(x - p.x_true)) / np.max(np.abs(p.x_true))
    fo = np.max(np.abs(x_ref - p.x_true)) / np.max(np.abs(p.x_true))
    log(f"  ferr gpu {fe:.2e} oracle {fo:.2e}")
    assert fe <= 10 * fo + 10 * n * U64


@pytest.mark.parametrize("n,kappa,seed,k", [(200, 1e8, 4, 5), (256, 1e9, 2, 8)])
def test_uniform_products_shared_factors(lib, n, kappa, seed, k):
    p = randsvd_problem(n, kappa, seed)
    o = oracle_options(uf="fp32", u="fp64", ur="dd", m=20, k=k, tau=1e-8, matvec="u")
    f = refine.factor(p.a, o)
    x_ref, info_ref = refine.solve(f, p.b)
    log(f"[uniform-shared] n={n} kappa={kappa:g}")
    h = lib.import_factors(_dev(p.a), _dev(encode_factors(f.lu, "fp32")),
                           f.ipiv.astype(np.int32), f.e, **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    _compare(p, x_ref, info_ref, x.cpu().numpy(), info, n, True)


@pytest.mark.parametrize("kind,n,m,k", [("randsvd", 300, 5, 2), ("prolate", 240, 6, 3)])
def test_uniform_products_full_path(lib, kind, n, m, k):
    p = prolate_problem(n, 0.48, seed=3) if kind == "prolate" else randsvd_problem(n, 1e8, 3)
    o = oracle_options(uf="fp32", u="fp64", ur="dd", m=m, k=k, tau=1e-8, matvec="u")
    x_ref, info_ref, _ = refine.gmresir(p.a, p.b, o)
    log(f"[uniform] {kind} n={n}")
    h = lib.factor(_dev(p.a), **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    _compare(p, x_ref, info_ref, x.cpu().numpy(), info, n, False)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_reuse_recycle_shared_factors(lib, seed):
    p = randsvd_problem(100, 1e4, seed)
    o = oracle_options(m=20, k=5, reuse=True)
    f = refine.factor(p.a, o)
    x_ref, info_ref = refine.solve(f, p.b)
    log(f"[reuse-shared] seed={seed}")
    h = lib.import_factors(_dev(p.a), _dev(encode_factors(f.lu, "fp16").view(np.int16)),
                           f.ipiv.astype(np.int32), f.e, **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    _compare(p, x_ref, info_ref, x.cpu().numpy(), info, 100, True)


@pytest.mark.parametrize("n,kappa,m,k", [(513, 1e4, 30, 10), (777, 1e4, 40, 8)])
def test_reuse_recycle_full_path(lib, n, kappa, m, k):
    p = randsvd_problem(n, kappa, 2)
    o = oracle_options(m=m, k=k, reuse=True)
    x_ref, info_ref, _ = refine.gmresir(p.a, p.b, o)
    log(f"[reuse] n={n}")
    h = lib.factor(_dev(p.a), **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    _compare(p, x_ref, info_ref, x.cpu().numpy(), info, n, False)


@pytest.mark.parametrize("k,seed", [(5, 1), (0, 2), (5, 3)])
def test_mgs_shared_factors(lib, k, seed):
    """opts.ortho = 1 (modified Gram-Schmidt, one basis column at a time) on
    the oracle's factors against the oracle's ortho = "mgs": counts within
    +-2 per step (the inner products are fp64 sums in another order)."""
    p = randsvd_problem(200, 1e4, seed)
    o = oracle_options(m=20, k=k, ortho="mgs")
    f = refine.factor(p.a, o)
    x_ref, info_ref = refine.solve(f, p.b)
    log(f"[mgs-shared] n=200 k={k} seed={seed}")
    h = lib.import_factors(_dev(p.a), _dev(encode_factors(f.lu, "fp16").view(np.int16)),
                           f.ipiv.astype(np.int32), f.e, **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    _compare(p, x_ref, info_ref, x.cpu().numpy(), info, 200, False)


def test_mgs_full_path_ragged(lib):
    p = randsvd_problem(513, 1e4, 2)
    o = oracle_options(m=30, k=10, ortho="mgs")
    x_ref, info_ref, _ = refine.gmresir(p.a, p.b, o)
    log("[mgs-full] n=513")
    h = lib.factor(_dev(p.a), **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    _compare(p, x_ref, info_ref, x.cpu().numpy(), info, 513, False)
