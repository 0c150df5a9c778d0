"""GPU checks of the per-solve record and the error report (the error
measures of Table 2), of the differentiable solve's status reporting, and of
the recycle state after the automatic choice of k.

* gmresir_errors: normwise and componentwise backward errors from a
  double-double residual and the forward error, against the same measures
  computed on the host with the oracle's double-double product;
* the record's componentwise backward error is never below the normwise one
  (each denominator (|A||x| + |b|)_i is at most ||A||_inf ||x||_inf +
  ||b||_inf), and both end below the target; the phase timers are
  non-negative and cover the solve;
* a forward solve that ends ENOCONV raises through the autograd Function and
  carries its record;
* after gmresir_choose_k a kept recycle space is dropped: the next solve is
  bit-identical to the first solve on a fresh handle.
"""
import numpy as np
import pytest

from gpu_util import U64, log
from oracle import fp
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


def _host_errors(a, b, x, x_true):
    rh, rl = fp.dd_gemv(a, x, y0h=b, y0l=np.zeros_like(b), sign=-1.0)
    r = rh + rl
    nw = np.max(np.abs(r)) / (np.max(np.sum(np.abs(a), axis=1)) * np.max(np.abs(x))
                              + np.max(np.abs(b)))
    den = np.abs(a) @ np.abs(x) + np.abs(b)
    cw = np.max(np.where(r == 0, 0.0, np.abs(r) / den))
    fe = np.max(np.abs(x - x_true)) / np.max(np.abs(x_true))
    return nw, cw, fe


@pytest.mark.parametrize("n,u,ur", [(200, "fp32", "fp64"), (257, "fp32", "dd"),
                                    (130, "fp64", "dd")])
def test_error_report_and_record(lib, n, u, ur):
    p = randsvd_problem(n, 1e3, 5)
    tau = 1e-4 if u == "fp32" else 1e-8
    uf = "fp16" if u == "fp32" else "fp32"
    log(f"[record] n={n} ({uf}, {u}, {ur})")
    h = lib.factor(_dev(p.a), uf=uf, u=u, ur=ur, m=20, k=5, tau=tau)
    x, info = h.solve(_dev(p.b))
    assert info["status"] == 0
    nw, cw, fe = h.errors(_dev(p.b), x, _dev(p.x_true))
    nw2, cw2, fe2 = h.errors(_dev(p.b), x)
    h.free()
    xh = x.cpu().numpy()
    rnw, rcw, rfe = _host_errors(p.a, p.b, xh, p.x_true)
    log(f"[record] gpu {nw:.3e} {cw:.3e} {fe:.3e} host {rnw:.3e} {rcw:.3e} {rfe:.3e}")
    assert abs(nw - rnw) <= 1e-10 * rnw + 1e-300
    assert abs(cw - rcw) <= 1e-10 * rcw + 1e-300
    assert abs(fe - rfe) <= 1e-12 * rfe
    assert nw2 == nw and cw2 == cw and np.isnan(fe2)
    # the record
    steps = info["steps"]
    assert len(info["berr_cw"]) == steps + 1
    for a, c in zip(info["berr"], info["berr_cw"]):
        assert c >= a * (1 - 1e-12)
    assert info["berr"][-1] <= 1e-14 and info["berr_cw"][-1] >= info["berr"][-1]
    t = [info[k] for k in ("t_x0_s", "t_residual_s", "t_precond_s", "t_recycle_s",
                           "t_arnoldi_s")]
    log(f"[record] phases {['%.2e' % v for v in t]} solve {info['t_solve_s']:.2e}")
    assert all(v >= 0 for v in t)
    assert sum(t) <= info["t_solve_s"] * 1.05 + 1e-4
    assert sum(t) >= 0.3 * info["t_solve_s"]
    assert t[2] > 0 and t[4] > 0


def test_gradient_raises_on_enoconv(lib):
    from paper_2201_09827_amd import GmresirError
    from paper_2201_09827_amd import autograd as ga
    p = randsvd_problem(128, 1e7, 2)
    a = _dev(p.a).requires_grad_(True)
    b = _dev(p.b).requires_grad_(True)
    rec = {}
    log("[grad-status] n=128 kappa=1e7 imax=1")
    with pytest.raises(GmresirError) as ei:
        ga.solve(a, b, records=rec, m=10, k=2, imax=1)
    assert ei.value.status == 3
    assert ei.value.info["status"] == 3 and rec["forward"]["status"] == 3
    # a solvable system passes and reports both records
    p = randsvd_problem(64, 1e2, 3)
    a = _dev(p.a).requires_grad_(True)
    b = _dev(p.b).requires_grad_(True)
    rec = {}
    x = ga.solve(a, b, records=rec, m=10, k=2)
    (0.5 * torch.sum(x * x)).backward()
    assert rec["forward"]["status"] == 0 and rec["adjoint"]["status"] == 0


def test_choose_k_drops_the_kept_space(lib):
    p = randsvd_problem(300, 1e4, 4)
    kw = dict(m=20, k=6, keep_recycle=1, reuse_recycle=1)
    log("[choose-k-state] n=300")
    h0 = lib.factor(_dev(p.a), **kw)
    x0, i0 = h0.solve(_dev(p.b))
    h0.free()
    h = lib.factor(_dev(p.a), **kw)
    _, i1 = h.solve(_dev(p.b))          # leaves a kept space
    assert i1["recycle_dim"] > 0
    kb, its, st = h.choose_k(_dev(p.b), 6)
    x2, i2 = h.solve(_dev(p.b))          # must start without one
    h.free()
    assert i2["its"] == i0["its"] and i2["steps"] == i0["steps"]
    assert torch.equal(x2, x0)
    assert i2["berr"][-1] <= 1e-14 and i2["berr"][-1] <= 8 * 300 * U64


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_recycle_setup_by_householder_qr(lib, monkeypatch, seed):
    """The branch a CholeskyQR2 breakdown takes (Householder QR of A-tilde U_k
    on the host, forced through the library's test hook): with the oracle's
    own factors every count must equal the oracle's, whose recycle set-up is
    that same Householder QR."""
    from gpu_util import encode_factors, lib_options, oracle_options
    from oracle import refine
    p = randsvd_problem(100, 1e4, seed)
    o = oracle_options(m=20, k=5)
    f = refine.factor(p.a, o)
    x_ref, info_ref = refine.solve(f, p.b)
    monkeypatch.setenv("GMRESIR_RECYCLE_QR", "householder")
    log(f"[recycle-hqr] seed={seed}")
    h = lib.import_factors(_dev(p.a), _dev(encode_factors(f.lu, "fp16").view(np.int16)),
                           f.ipiv.astype(np.int32), f.e, **lib_options(o))
    x, info = h.solve(_dev(p.b))
    h.free()
    log(f"[recycle-hqr] oracle its={info_ref.its} gpu its={info['its']}")
    assert info_ref.steps >= 2 and info["status"] == 0
    assert info["steps"] == info_ref.steps and info["its"] == info_ref.its
    assert info["berr"][-1] <= 8 * 100 * U64
    fe = np.max(np.abs(x.cpu().numpy() - p.x_true)) / np.max(np.abs(p.x_true))
    fo = np.max(np.abs(x_ref - p.x_true)) / np.max(np.abs(p.x_true))
    assert fe <= 10 * fo + 1000 * U64


@pytest.mark.parametrize("n,k", [(1000, 10), (4097, 5), (300, 0)])
def test_fused_product_and_lower_solve_match_separate_launches(lib, monkeypatch, n, k):
    """The Arnoldi step's A_u product fused into the lower solve's launch
    (the default) against the separate launches (GMRESIR_FUSED_ATILDE=0):
    the same sums in the same order, so every count and every bit of x must
    agree."""
    p = randsvd_problem(n, 1e3, 7)
    a, b = _dev(p.a), _dev(p.b)
    log(f"[fused] n={n} k={k}")
    h = lib.factor(a, m=20, k=k)
    x1, i1 = h.solve(b)
    h.free()
    monkeypatch.setenv("GMRESIR_FUSED_ATILDE", "0")
    h = lib.factor(a, m=20, k=k)
    x0, i0 = h.solve(b)
    h.free()
    log(f"[fused] its fused {i1['its']} separate {i0['its']}")
    assert i1["status"] == i0["status"] == 0
    assert i1["its"] == i0["its"] and i1["berr"] == i0["berr"]
    assert torch.equal(x1, x0)


def test_caller_allocator_hooks(lib):
    """opts.alloc / opts.free_ route every device buffer of a handle through
    the caller's allocator (here torch's caching allocator): the solve is
    bit-identical to the one on the library's own memory, and gmresir_free
    hands every block back.  An allocator that fails gives ENOMEM."""
    p = randsvd_problem(700, 1e3, 9)
    a, b = _dev(p.a), _dev(p.b)
    log("[alloc-hooks] n=700")
    h = lib.factor(a, m=20, k=5)
    x0, i0 = h.solve(b)
    h.free()
    al = lib.TorchAllocator()
    h = lib.factor(a, m=20, k=5, **al.opts())
    x1, i1 = h.solve(b)
    assert al.calls > 0 and len(al.live) > 0
    h.free()
    assert len(al.live) == 0
    assert i1["its"] == i0["its"] and torch.equal(x1, x0)

    def refuse(nbytes, user):
        return None

    def nothing(ptr, user):
        pass

    ra = lib._ALLOC_FN(refuse)
    rf = lib._FREE_FN(nothing)
    import ctypes
    with pytest.raises(lib.GmresirError) as ei:
        lib.factor(a, m=20, k=5, alloc=ctypes.cast(ra, ctypes.c_void_p).value,
                   free_=ctypes.cast(rf, ctypes.c_void_p).value)
    assert ei.value.status == -2
