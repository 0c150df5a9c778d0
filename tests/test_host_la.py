"""The library's host small-problem routines (host_la.cpp: Givens least
squares, thin QR, Cholesky, triangular inverse, the real eigenproblem and the
harmonic Ritz vectors of GCRO-DR), built on the CPU with g++ under the
address and undefined-behaviour sanitizers and checked against numpy/scipy:

* givens_lsq against numpy.linalg.lstsq on the same (j+1) x j Hessenberg
  matrix (the GMRES least-squares problem of Section 2);
* qr_thin against numpy's QR (signs normalised to a non-negative diagonal of
  R), and its rank-deficiency report;
* cholesky_upper and inv_upper against numpy;
* eig_real against numpy.linalg.eigvals, with the eigenvector residual;
* harmonic_ritz against scipy.linalg.eig on G^T G z = theta G^T M z: the
  span of the returned columns equals the span of the eigenvectors of the k
  smallest |theta| (the recycle-space refresh of GCRO-DR, Section 2).

The sanitizer build aborts on any out-of-bounds access, leak or undefined
behaviour, so every call here also checks the routines' memory use.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.linalg as sla

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2201_09827_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "host", "host_la_driver.cpp")


@pytest.fixture(scope="module")
def driver():
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    d = tempfile.mkdtemp(prefix="host_la_")
    exe = os.path.join(d, "host_la_driver")
    cmd = [gxx, "-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", f"-I{CSRC}",
           DRIVER, os.path.join(CSRC, "host_la.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def _call(exe, lines):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         env=env, timeout=120)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr, res.stderr[-4000:]
    return [np.array([float(t) for t in ln.split()]) for ln in res.stdout.strip().splitlines()]


def _fmt(*parts):
    out = []
    for p in parts:
        if isinstance(p, np.ndarray):
            out.extend(f"{v:.17g}" for v in p.ravel(order="F"))
        else:
            out.append(str(p))
    return " ".join(out)


def test_givens_least_squares(driver):
    g = np.random.default_rng(1)
    cases, refs = [], []
    for j in (1, 2, 5, 17, 30):
        ldh = j + 3
        H = np.zeros((ldh, j))
        hb = np.triu(g.standard_normal((j + 1, j)), -1)
        H[: j + 1] = hb
        beta = float(g.uniform(0.5, 2.0))
        cases.append(_fmt("givens", j, ldh, f"{beta:.17g}", H))
        rhs = np.zeros(j + 1)
        rhs[0] = beta
        y, *_ = np.linalg.lstsq(hb, rhs, rcond=None)
        refs.append((y, np.linalg.norm(rhs - hb @ y)))
    for out, (y, res) in zip(_call(driver, cases), refs):
        assert abs(out[0] - res) <= 1e-12 * max(1.0, res)
        np.testing.assert_allclose(out[1:], y, rtol=1e-10, atol=1e-12)


def test_qr_thin(driver):
    g = np.random.default_rng(2)
    cases, refs = [], []
    for m, k in ((5, 1), (8, 8), (40, 11), (100, 30)):
        A = g.standard_normal((m, k))
        cases.append(_fmt("qr", m, k, A))
        q, r = np.linalg.qr(A)
        s = np.sign(np.diag(r))
        refs.append((m, k, A, q * s, s[:, None] * r))
    # rank deficient: a repeated column
    A = g.standard_normal((10, 4))
    A[:, 2] = A[:, 1]
    cases.append(_fmt("qr", 10, 4, A))
    outs = _call(driver, cases)
    for out, (m, k, A, q, r) in zip(outs, refs):
        assert out[0] == 1
        Q = out[1:1 + m * k].reshape((m, k), order="F")
        R = out[1 + m * k:].reshape((k, k), order="F")
        np.testing.assert_allclose(Q, q, atol=1e-12)
        np.testing.assert_allclose(R, r, atol=1e-12 * np.abs(r).max())
        assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)
    assert outs[-1][0] == 0


def test_cholesky_and_triangular_inverse(driver):
    g = np.random.default_rng(3)
    cases, refs = [], []
    for k in (1, 3, 12):
        X = g.standard_normal((k + 4, k))
        G = X.T @ X
        cases.append(_fmt("chol", k, G))
        refs.append(("chol", k, np.linalg.cholesky(G).T))
        R = np.triu(g.standard_normal((k, k))) + 3 * np.eye(k)
        cases.append(_fmt("invu", k, R))
        refs.append(("invu", k, np.linalg.inv(R)))
    cases.append(_fmt("chol", 2, np.array([[1.0, 2.0], [2.0, 1.0]])))   # indefinite
    outs = _call(driver, cases)
    for out, (kind, k, ref) in zip(outs, refs):
        if kind == "chol":
            assert out[0] == 1
            np.testing.assert_allclose(out[1:].reshape((k, k), order="F"), ref, rtol=1e-12,
                                       atol=1e-12)
        else:
            np.testing.assert_allclose(out.reshape((k, k), order="F"), ref, rtol=1e-10,
                                       atol=1e-12)
    assert outs[-1][0] == 0


def _eig_out(out, N):
    w = out[1:1 + 2 * N].reshape(N, 2)
    w = w[:, 0] + 1j * w[:, 1]
    v = out[1 + 2 * N:].reshape(N * N, 2)
    V = (v[:, 0] + 1j * v[:, 1]).reshape((N, N), order="F")
    return w, V


def test_real_eigenproblem(driver):
    g = np.random.default_rng(4)
    cases, mats = [], []
    for N in (1, 2, 6, 20, 51):
        A = g.standard_normal((N, N))
        cases.append(_fmt("eig", N, A))
        mats.append(A)
    # structured cases reaching every branch of the real Schur solver: all
    # eigenvalues real (symmetric), already triangular, a repeated
    # eigenvalue, a companion matrix with complex roots, the zero matrix
    S = g.standard_normal((12, 12))
    extra = [S + S.T, np.triu(g.standard_normal((7, 7)))]
    Qr, _ = np.linalg.qr(g.standard_normal((5, 5)))
    extra.append(Qr @ np.diag([2.0, 2.0, 3.0, -1.0, 2.0]) @ Qr.T)
    C = np.zeros((6, 6))
    C[1:, :-1] = np.eye(5)
    C[:, -1] = -np.array([1.0, 0.0, 2.0, 0.0, 3.0, 1.0])
    extra += [C, np.zeros((3, 3))]
    for A in extra:
        cases.append(_fmt("eig", A.shape[0], A))
        mats.append(A)
    # a matrix with a known spectrum: block diagonal rotation-scalings
    B = np.zeros((4, 4))
    B[:2, :2] = [[1.0, -2.0], [2.0, 1.0]]
    B[2:, 2:] = [[3.0, 0.0], [0.0, -0.5]]
    Qm, _ = np.linalg.qr(g.standard_normal((4, 4)))
    A = Qm @ B @ Qm.T
    cases.append(_fmt("eig", 4, A))
    mats.append(A)
    for out, A in zip(_call(driver, cases), mats):
        N = A.shape[0]
        assert out[0] == 1
        w, V = _eig_out(out, N)
        ref = np.linalg.eigvals(A)
        key = lambda z: (round(z.real, 8), round(z.imag, 8))
        np.testing.assert_allclose(sorted(w, key=key), sorted(ref, key=key), atol=1e-9 *
                                   max(1.0, np.abs(ref).max()))
        res = np.abs(A @ V - V * w[None, :]).max()
        assert res <= 1e-9 * np.abs(A).max() * max(1.0, np.abs(V).max())
    w, _ = _eig_out(_call(driver, [cases[-1]])[0], 4)
    np.testing.assert_allclose(sorted(w, key=key), sorted([1 + 2j, 1 - 2j, 3, -0.5], key=key),
                               atol=1e-12)


def _span_distance(P, Z):
    """sin of the largest principal angle between span(P) and span(Z)."""
    qp, _ = np.linalg.qr(P)
    qz, _ = np.linalg.qr(Z)
    s = np.linalg.svd(qp.T @ qz, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - min(s) ** 2)))


@pytest.mark.parametrize("cols,k,seed", [(10, 3, 5), (20, 5, 6), (31, 10, 7), (8, 8, 8)])
def test_harmonic_ritz_vectors(driver, cols, k, seed):
    g = np.random.default_rng(seed)
    rows = cols + 1
    # the first-cycle form: G = Hbar (upper Hessenberg), M = [I; 0]
    G = np.triu(g.standard_normal((rows, cols)), -1)
    M = np.zeros((rows, cols))
    M[:cols] = np.eye(cols)
    out = _call(driver, [_fmt("hritz", rows, cols, k, G, M)])[0]
    kout = int(out[0])
    P = out[1:].reshape((cols, kout), order="F")
    theta, Z = sla.eig(G.T @ G, G.T @ M)
    order = np.argsort(np.abs(theta), kind="stable")
    # the reference basis: the same count of smallest |theta|, pairs as
    # (Re, Im) columns
    cols_ref = []
    used = set()
    for i in order:
        if len(cols_ref) >= kout:
            break
        if i in used:
            continue
        used.add(i)
        z = Z[:, i]
        if abs(theta[i].imag) > 1e-10 * abs(theta[i]):
            j = min((t for t in order if t not in used),
                    key=lambda t: abs(theta[t] - np.conj(theta[i])))
            used.add(j)
            cols_ref += [z.real, z.imag]
        else:
            cols_ref.append((z * np.exp(-1j * np.angle(z[np.argmax(np.abs(z))]))).real)
    Zr = np.column_stack(cols_ref[:kout])
    assert k - 1 <= kout <= k
    assert _span_distance(P, Zr) <= 1e-7
