"""A GMRES cycle's Arnoldi steps in one persistent launch (u = fp32,
classical Gram-Schmidt twice, n <= 8192) against the separate launches of
each step (GMRESIR_PERSISTENT=0 at handle creation).  The persistent kernel
forms every sum of the step -- the product with A_u, the two blocked
triangular solves, the three Gram-Schmidt passes with their per-block sums
paired and the 256-row chunks added in order, the Givens update -- in the
order the separate launches form it, so every count and every bit of x must
agree.  The timing class "arnoldi_cycle" shows that the persistent launch
ran (and that it did not where the shape is outside its limits).
"""
import numpy as np
import pytest

from gpu_util import log
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


def _cycles(h):
    for s in h.kernel_stats():
        if s["name"] == "arnoldi_cycle":
            return s["launches"]
    return 0


def _solve(lib, monkeypatch, a, bs, persistent, **kw):
    monkeypatch.setenv("GMRESIR_PERSISTENT", "1" if persistent else "0")
    h = lib.factor(a, timing=lib.timing_mask(["arnoldi_cycle"]), **kw)
    out = [h.solve(b) for b in bs]
    launches = _cycles(h)
    h.free()
    return out, launches


@pytest.mark.parametrize("n,k,m,kappa,uf", [(100, 0, 10, 1e2, "fp16"),
                                            (129, 3, 10, 1e3, "fp16"),
                                            (257, 5, 20, 1e3, "fp16"),
                                            (640, 8, 25, 1e5, "bf16"),
                                            (1036, 10, 30, 4.5e7, "fp16"),
                                            (1500, 6, 40, 1e4, "fp32"),
                                            (2048, 10, 30, 1e4, "fp16")])
def test_persistent_cycle_is_bit_identical(lib, monkeypatch, n, k, m, kappa, uf):
    p = randsvd_problem(n, kappa, 31)
    a, b = _dev(p.a), _dev(p.b)
    kw = dict(uf=uf, m=m, k=k, maxit=200)
    log(f"[cycle] n={n} k={k} m={m} kappa={kappa:g} uf={uf}")
    (r1,), c1 = _solve(lib, monkeypatch, a, [b], True, **kw)
    (r0,), c0 = _solve(lib, monkeypatch, a, [b], False, **kw)
    (x1, i1), (x0, i0) = r1, r0
    log(f"[cycle] its persistent {i1['its']} separate {i0['its']} launches {c1} / {c0}")
    assert c1 > 0 and c0 == 0
    assert i1["cycles_persistent"] > 0 and i1["cycles_fallback"] == 0
    assert i0["cycles_persistent"] == 0 and i0["cycles_fallback"] == 0
    assert i1["status"] == i0["status"]
    assert i1["its"] == i0["its"] and i1["berr"] == i0["berr"]
    assert i1["recycle_dim"] == i0["recycle_dim"]
    assert torch.equal(x1, x0)


@pytest.mark.parametrize("n,k", [(4097, 10), (8192, 10)])
def test_persistent_cycle_at_large_orders(lib, monkeypatch, n, k):
    """Orders beyond 4096 (up to 64 blocks per chain, rows of more than eight
    256-column pieces, exchanges over more than 16 blocks), among them the
    benchmark's n = 8192: the same bits as the separate launches."""
    from synthetic import randsvd_problem_torch
    a, _, b = randsvd_problem_torch(n, 1e2, 3)
    kw = dict(m=30, k=k, maxit=60)
    log(f"[cycle-large] n={n} k={k}")
    (r1,), c1 = _solve(lib, monkeypatch, a, [b], True, **kw)
    (r0,), c0 = _solve(lib, monkeypatch, a, [b], False, **kw)
    (x1, i1), (x0, i0) = r1, r0
    log(f"[cycle-large] its persistent {i1['its']} separate {i0['its']} launches {c1} / {c0}")
    assert c1 > 0 and c0 == 0 and i1["cycles_persistent"] > 0
    assert i1["status"] == i0["status"] == 0
    assert i1["its"] == i0["its"] and i1["berr"] == i0["berr"]
    assert torch.equal(x1, x0)


def test_persistent_cycle_with_kept_recycle_space(lib, monkeypatch):
    """Several right-hand sides with the recycle space carried over: every
    cycle's basis starts with C_k."""
    p = randsvd_problem(900, 1e4, 33)
    a = _dev(p.a)
    g = np.random.default_rng(7)
    bs = [_dev(p.a @ g.uniform(-1, 1, 900)) for _ in range(3)]
    log("[cycle-keep] n=900 k=6 m=20, three right-hand sides")
    r1, c1 = _solve(lib, monkeypatch, a, bs, True, m=20, k=6, keep_recycle=1)
    r0, c0 = _solve(lib, monkeypatch, a, bs, False, m=20, k=6, keep_recycle=1)
    assert c1 > 0 and c0 == 0
    for (x1, i1), (x0, i0) in zip(r1, r0):
        assert i1["its"] == i0["its"] and i1["recycle_dim"] == i0["recycle_dim"]
        assert torch.equal(x1, x0)


@pytest.mark.parametrize("n,u,extra", [(8193, "fp32", {}), (600, "fp64", {}),
                                        (600, "fp32", {"ortho": "mgs"})])
def test_persistent_cycle_outside_its_limits(lib, monkeypatch, n, u, extra):
    """Beyond n = 8192, for u = fp64 and with modified Gram-Schmidt the cycle
    runs as separate launches (no persistent launch is made)."""
    if n > 4096:
        from synthetic import randsvd_problem_torch
        a, _, b = randsvd_problem_torch(n, 1e2, 35)
    else:
        p = randsvd_problem(n, 1e3, 35)
        a, b = _dev(p.a), _dev(p.b)
    uf = "fp16" if u == "fp32" else "fp32"
    kw = dict(uf=uf, u=u, ur="dd" if u == "fp64" else "fp64", m=20, k=4,
              tau=1e-4 if u == "fp32" else 1e-8, **extra)
    log(f"[cycle-limits] n={n} u={u} {extra}")
    (r,), c = _solve(lib, monkeypatch, a, [b], True, **kw)
    assert c == 0 and r[1]["status"] == 0


def test_persistent_cycle_that_gives_up_falls_back(lib, monkeypatch):
    """A persistent launch whose workgroups are not all resident together
    gives up before writing anything and the cycle runs as separate
    launches.  Forced from the host with a zero arrival bound
    (GMRESIR_CYCLE_ARRIVE_US=0: the first workgroup to arrive gives up, and
    every kernel still ends normally): the results must equal those of the
    separate launches, and no persistent launch is counted."""
    p = randsvd_problem(700, 1e4, 37)
    a, b = _dev(p.a), _dev(p.b)
    kw = dict(m=20, k=5, maxit=100)
    log("[cycle-fallback] n=700 arrival bound 0")
    monkeypatch.setenv("GMRESIR_CYCLE_ARRIVE_US", "0")
    (r1,), c1 = _solve(lib, monkeypatch, a, [b], True, **kw)
    monkeypatch.delenv("GMRESIR_CYCLE_ARRIVE_US")
    (r0,), c0 = _solve(lib, monkeypatch, a, [b], False, **kw)
    (x1, i1), (x0, i0) = r1, r0
    log(f"[cycle-fallback] its {i1['its']} / {i0['its']} launches {c1} / {c0}")
    assert c1 == 0 and c0 == 0
    assert i1["cycles_fallback"] > 0 and i1["cycles_persistent"] == 0
    assert i1["status"] == i0["status"] and i1["its"] == i0["its"]
    assert i1["berr"] == i0["berr"] and torch.equal(x1, x0)
