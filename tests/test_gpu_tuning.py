"""The Arnoldi step's orthogonalisation in one single-workgroup launch
(classical Gram-Schmidt twice, the Hessenberg column with its Givens
rotation, and the normalisation of the next basis vector) against the three
multi-workgroup passes and the separate normalisation: both form every sum
in the same order, so every count and every bit of x must agree.  The
library picks one of the two by timing them (the autotuner); the variant is
forced here with GMRESIR_ORTHO_SMALL at handle creation, and the default
(tuned) handle must agree with both.  The cycle's persistent single launch
(the default where the shape allows it) is switched off here
(GMRESIR_PERSISTENT=0), so that these are the separate launches.
"""
import numpy as np
import pytest

from gpu_util import log
from synthetic import randsvd_problem

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _separate_launches(monkeypatch):
    monkeypatch.setenv("GMRESIR_PERSISTENT", "0")


@pytest.fixture(scope="module")
def lib():
    import paper_2201_09827_amd as g
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g.load_library()
    return g


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _solve(lib, monkeypatch, a, b, variant, **kw):
    if variant is None:
        monkeypatch.delenv("GMRESIR_ORTHO_SMALL", raising=False)
    else:
        monkeypatch.setenv("GMRESIR_ORTHO_SMALL", variant)
    h = lib.factor(a, **kw)
    x, info = h.solve(b)
    h.free()
    return x, info


@pytest.mark.parametrize("n,k,kappa,u,ur", [(100, 5, 1e3, "fp32", "fp64"),
                                            (257, 0, 1e3, "fp32", "fp64"),
                                            (1000, 10, 1e5, "fp32", "fp64"),
                                            (2048, 10, 1e4, "fp32", "fp64"),
                                            (4096, 8, 1e3, "fp32", "fp64"),
                                            (600, 6, 1e6, "fp64", "dd")])
def test_single_launch_orthogonalisation_is_bit_identical(lib, monkeypatch, n, k, kappa, u, ur):
    p = randsvd_problem(n, kappa, 13)
    a, b = _dev(p.a), _dev(p.b)
    uf = "fp16" if u == "fp32" else "fp32"
    tau = 1e-4 if u == "fp32" else 1e-8
    kw = dict(uf=uf, u=u, ur=ur, m=25, k=k, tau=tau)
    log(f"[ortho-small] n={n} k={k} kappa={kappa:g} ({uf}, {u}, {ur})")
    x0, i0 = _solve(lib, monkeypatch, a, b, "0", **kw)
    x1, i1 = _solve(lib, monkeypatch, a, b, "1", **kw)
    xt, it = _solve(lib, monkeypatch, a, b, None, **kw)
    log(f"[ortho-small] its multi {i0['its']} single {i1['its']} tuned {it['its']}")
    assert i0["status"] == i1["status"] == it["status"]
    assert i0["its"] == i1["its"] == it["its"]
    assert i0["berr"] == i1["berr"] == it["berr"]
    assert torch.equal(x0, x1) and torch.equal(x0, xt)


def test_single_launch_with_kept_recycle_space(lib, monkeypatch):
    """Several right-hand sides with the recycle space carried over (the
    basis then starts with C_k in every cycle)."""
    p = randsvd_problem(700, 1e4, 21)
    a = _dev(p.a)
    g = np.random.default_rng(5)
    bs = [_dev(p.a @ g.uniform(-1, 1, 700)) for _ in range(3)]
    res = {}
    for v in ("0", "1"):
        monkeypatch.setenv("GMRESIR_ORTHO_SMALL", v)
        h = lib.factor(a, m=20, k=6, keep_recycle=1)
        res[v] = [h.solve(b) for b in bs]
        h.free()
    for (x0, i0), (x1, i1) in zip(res["0"], res["1"]):
        assert i0["its"] == i1["its"] and i0["recycle_dim"] == i1["recycle_dim"]
        assert torch.equal(x0, x1)


@pytest.mark.parametrize("n,k", [(257, 5), (384, 0), (1000, 10), (4097, 8)])
def test_first_pass_inside_the_upper_solve_is_bit_identical(lib, monkeypatch, n, k):
    """The Arnoldi step's first Gram-Schmidt pass formed inside the upper
    triangular solve (the default with the multi-workgroup passes) against
    the separate pass (GMRESIR_FUSED_DOTS=0): the per-block sums are paired
    and the 256-row chunks added in the separate pass's order, so every
    count and every bit of x must agree (odd and even block counts)."""
    p = randsvd_problem(n, 1e4, 17)
    a, b = _dev(p.a), _dev(p.b)
    kw = dict(m=25, k=k)
    monkeypatch.setenv("GMRESIR_ORTHO_SMALL", "0")
    log(f"[dots-fused] n={n} k={k}")
    x1, i1 = _solve(lib, monkeypatch, a, b, "0", **kw)
    monkeypatch.setenv("GMRESIR_FUSED_DOTS", "0")
    x0, i0 = _solve(lib, monkeypatch, a, b, "0", **kw)
    monkeypatch.delenv("GMRESIR_FUSED_DOTS")
    log(f"[dots-fused] its fused {i1['its']} separate {i0['its']}")
    assert i1["status"] == i0["status"]
    assert i1["its"] == i0["its"] and i1["berr"] == i0["berr"]
    assert torch.equal(x1, x0)
