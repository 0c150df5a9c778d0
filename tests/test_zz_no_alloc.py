"""The no-allocation entry point gmresir_errors_noalloc (static per-device
scratch, results in device memory) against gmresir_errors on a handle: the
three error measures must be identical, on two calls in a row with the second
on a smaller system (the static array keeps the first call's contents), and
sizes beyond the static limit must be rejected."""
import ctypes

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


def test_noalloc_errors_match_the_handle_report(lib):
    for n, kappa, seed in ((700, 1e4, 1), (130, 1e2, 2)):
        p = randsvd_problem(n, kappa, seed)
        a, b, xt = _dev(p.a), _dev(p.b), _dev(p.x_true)
        log(f"[noalloc] n={n}")
        h = lib.factor(a, m=20, k=5)
        x, info = h.solve(b)
        ref = h.errors(b, x, xt)
        ref_nt = h.errors(b, x)
        h.free()
        out = torch.full((3,), -1.0, dtype=torch.float64, device="cuda")
        lib.errors_noalloc(a, b, x, out, x_true=xt)
        got = out.cpu().numpy()
        lib.errors_noalloc(a, b, x, out)
        got_nt = out.cpu().numpy()
        log(f"[noalloc] n={n} handle {ref} static {got.tolist()}")
        assert got[0] == ref[0] and got[1] == ref[1] and got[2] == ref[2]
        assert got_nt[0] == ref_nt[0] and got_nt[1] == ref_nt[1] and np.isnan(got_nt[2])


def test_noalloc_rejects_out_of_range_arguments(lib):
    L = lib.load_library()
    dummy = torch.zeros(4, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(dummy.data_ptr())
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.gmresir_errors_noalloc(p, 16385, 16386, p, p, None, p, s) == -1
    assert L.gmresir_errors_noalloc(p, 2, 3, p, p, None, p, s) == -1       # odd lda
    assert L.gmresir_errors_noalloc(None, 2, 2, p, p, None, p, s) == -1
