"""The LU's block column launch with its folded parts (fp16 / bf16 factors):
the block column's workgroups form their rows' share of the previous step's
trailing update and, while the update is small enough, the block row's
triangular solve; the update tiles then solve their own columns of the block
row and the last tile of each strip writes it back.  Every entry is formed
as the separate launches form it (the same matrix-core instruction over the
same k steps at the same position in its 32 x 32 block, the same order of
fused multiply-adds in the solve), so the exported factors must agree bit
for bit with GMRESIR_LU_FOLD=0 at handle creation, which keeps the separate
launches.  The orders cover one, two and many workgroups per block column (up to the
exchange's 32 at n = 16384),
block counts that are not multiples of the tile grid, both fold forms (the
solve moves in only once the update has at most 5.5 rounds of tiles over the
compute units: at n = 8192 from step 54 on) and a final partial block
column.
"""
import pytest

from gpu_util import log
from synthetic import randsvd_problem_torch

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2201_09827_amd as g
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g.load_library()
    return g


def _factors(lib, monkeypatch, a, uf, fold):
    monkeypatch.setenv("GMRESIR_LU_FOLD", "1" if fold else "0")
    h = lib.factor(a, uf=uf, u="fp32", ur="fp64", m=30, k=10)
    assert h.status == 0
    lu, ipiv, e = h.export_factors()
    h.free()
    return lu, ipiv, e


@pytest.mark.parametrize("n,uf", [(300, "fp16"), (700, "bf16"), (1100, "fp16"),
                                  (3000, "bf16"), (4800, "fp16"), (8192, "fp16"),
                                  (16384, "bf16")])
def test_folded_block_column_factors_bit_identical(lib, monkeypatch, n, uf):
    log(f"lu fold n={n} uf={uf}")
    a, _, _ = randsvd_problem_torch(n, 1e6, 7, device="cuda")
    lu1, p1, e1 = _factors(lib, monkeypatch, a, uf, True)
    lu0, p0, e0 = _factors(lib, monkeypatch, a, uf, False)
    assert e1 == e0
    assert (p1 == p0).all()
    diff = int((lu1 != lu0).sum())
    assert diff == 0, f"{diff} factor entries differ"
