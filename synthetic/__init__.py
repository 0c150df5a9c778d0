"""Seeded synthetic inputs for the mixed-precision GMRES-IR solvers.

This module is shared by the CPU oracle and by the GPU path.  It only draws
random numbers and builds the test matrices the paper uses; it contains none
of the solver's arithmetic (no rounding to low precision, no factorisation,
no Krylov method).

Matrices (Section 3 of the paper, the experimental setup):

* ``randsvd``: dense A = U diag(sigma) V^T with U, V Haar-distributed
  orthogonal matrices and geometrically spaced singular values from 1 down to
  1/kappa (MATLAB's randsvd "mode 3").  The paper draws them with MATLAB's
  generator, which cannot be reproduced here; this version draws U and V as
  the Q factor of a QR factorisation of a Gaussian matrix with the signs of
  R's diagonal moved into Q (Mezzadri 2007), which makes Q Haar distributed.
* ``prolate``: the symmetric Toeplitz prolate matrix with parameter w:
  a_ii = 2w and a_ij = sin(2 pi w (i - j)) / (pi (i - j)).

Right-hand sides: the paper uses b = ones; the benchmark workloads use a known
solution x_true (uniform on [-1, 1] or standard normal) and b = A x_true
computed in float64.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "generator",
    "haar_orthogonal",
    "randsvd_singular_values",
    "randsvd",
    "prolate",
    "uniform_vector",
    "normal_vector",
    "rhs_from_solution",
    "Problem",
    "randsvd_problem",
    "prolate_problem",
    "randsvd_problem_torch",
]


def generator(seed: int) -> np.random.Generator:
    """PCG64 generator for ``seed`` (every input in this project is seeded)."""
    return np.random.Generator(np.random.PCG64(int(seed)))


def haar_orthogonal(n: int, g: np.random.Generator) -> np.ndarray:
    """Haar-distributed n x n orthogonal matrix (QR of a Gaussian, sign fix)."""
    z = g.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def randsvd_singular_values(n: int, kappa: float) -> np.ndarray:
    """Geometrically spaced singular values sigma_i = kappa^(-(i-1)/(n-1))."""
    if n == 1:
        return np.ones(1)
    i = np.arange(n, dtype=np.float64)
    return np.power(float(kappa), -i / (n - 1))


def randsvd(n: int, kappa: float, seed: int) -> np.ndarray:
    """Dense randsvd mode-3 matrix, float64, C-contiguous (row-major).

    U is drawn first, then V, from one generator seeded with ``seed``.
    """
    g = generator(seed)
    u = haar_orthogonal(n, g)
    v = haar_orthogonal(n, g)
    sigma = randsvd_singular_values(n, kappa)
    return np.ascontiguousarray((u * sigma[None, :]) @ v.T)


def prolate(n: int, w: float) -> np.ndarray:
    """Prolate Toeplitz matrix of order n with parameter w (0 < w < 1/2)."""
    k = np.arange(n, dtype=np.float64)
    col = np.empty(n)
    col[0] = 2.0 * w
    col[1:] = np.sin(2.0 * np.pi * w * k[1:]) / (np.pi * k[1:])
    idx = np.abs(np.subtract.outer(np.arange(n), np.arange(n)))
    return np.ascontiguousarray(col[idx])


def uniform_vector(n: int, g: np.random.Generator) -> np.ndarray:
    return g.uniform(-1.0, 1.0, size=n)


def normal_vector(n: int, g: np.random.Generator) -> np.ndarray:
    return g.standard_normal(n)


def rhs_from_solution(a: np.ndarray, x_true: np.ndarray) -> np.ndarray:
    """b = A x_true in float64 (plain BLAS product)."""
    return np.ascontiguousarray(a @ x_true)


class Problem:
    """A seeded linear system: matrix, known solution and right-hand side."""

    def __init__(self, name: str, a: np.ndarray, x_true: np.ndarray | None,
                 b: np.ndarray):
        self.name = name
        self.a = a
        self.x_true = x_true
        self.b = b

    @property
    def n(self) -> int:
        return self.a.shape[0]


def randsvd_problem(n: int, kappa: float, seed: int) -> Problem:
    """randsvd mode-3 system with x_true ~ U(-1, 1) and b = A x_true.

    The generator state after drawing U and V draws x_true, so one seed
    determines the whole system.
    """
    g = generator(seed)
    u = haar_orthogonal(n, g)
    v = haar_orthogonal(n, g)
    sigma = randsvd_singular_values(n, kappa)
    a = np.ascontiguousarray((u * sigma[None, :]) @ v.T)
    x = uniform_vector(n, g)
    return Problem(f"randsvd(n={n},kappa={kappa:g},seed={seed})", a, x,
                   rhs_from_solution(a, x))


def prolate_problem(n: int, w: float, seed: int | None = None) -> Problem:
    """Prolate system; b = ones when ``seed`` is None (the paper's choice),
    else x_true ~ N(0, 1) from ``seed`` and b = A x_true."""
    a = prolate(n, w)
    if seed is None:
        return Problem(f"prolate(n={n},w={w:g},b=ones)", a, None, np.ones(n))
    g = generator(seed)
    x = normal_vector(n, g)
    return Problem(f"prolate(n={n},w={w:g},seed={seed})", a, x,
                   rhs_from_solution(a, x))


def randsvd_problem_torch(n: int, kappa: float, seed: int, device="cuda"):
    """randsvd mode-3 system drawn with torch on ``device`` (same recipe as
    :func:`randsvd_problem`: Haar U then V from the QR of Gaussian matrices
    with R's diagonal signs moved into Q, geometric singular values,
    x_true ~ U(-1, 1), b = A x_true in float64).  A different random stream
    from the numpy version; used where generating n ~ 1e4 on the CPU would
    dominate the run.  Returns float64 tensors (a, x_true, b) on ``device``.
    """
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))

    def haar():
        z = torch.randn((n, n), generator=gen, dtype=torch.float64, device=device)
        q, r = torch.linalg.qr(z)
        s = torch.sign(torch.diagonal(r))
        s[s == 0] = 1.0
        return q * s[None, :]

    u = haar()
    v = haar()
    sigma = torch.from_numpy(randsvd_singular_values(n, kappa)).to(device)
    a = (u * sigma[None, :]) @ v.T.contiguous()
    del u, v
    x = torch.rand(n, generator=gen, dtype=torch.float64, device=device) * 2.0 - 1.0
    b = a @ x
    return a.contiguous(), x, b


def prolate_problem_torch(n: int, w: float, seed: int, device="cuda"):
    """Prolate system assembled on ``device``: the Toeplitz matrix of
    :func:`prolate` (first column computed in numpy, entries gathered by
    |i - j| in row blocks), x_true ~ N(0, 1) from the numpy generator seeded
    with ``seed`` (the same x_true as :func:`prolate_problem`), b = A x_true in
    float64 on the device.  Returns float64 tensors (a, x_true, b)."""
    import torch
    k = np.arange(n, dtype=np.float64)
    col = np.empty(n)
    col[0] = 2.0 * w
    col[1:] = np.sin(2.0 * np.pi * w * k[1:]) / (np.pi * k[1:])
    colt = torch.from_numpy(col).to(device)
    a = torch.empty((n, n), dtype=torch.float64, device=device)
    j = torch.arange(n, device=device)
    step = 1024
    for r0 in range(0, n, step):
        i = torch.arange(r0, min(n, r0 + step), device=device)
        a[r0:r0 + i.numel()] = colt[torch.abs(i[:, None] - j[None, :])]
    x = torch.from_numpy(normal_vector(n, generator(seed))).to(device)
    b = a @ x
    return a, x, b


def batch_specs(count: int, seed: int, n_range=(128, 2048), log10_kappa=(1.0, 8.0),
                nrhs_range=(1, 8)):
    """Specifications of a batch of independent randsvd systems of uneven
    size: n uniform on the integers of ``n_range``, log10 kappa_2 uniform on
    ``log10_kappa``, the number of right-hand sides uniform on the integers of
    ``nrhs_range``.  Returns a list of dicts (n, kappa, nrhs, seed) with one
    derived seed per system."""
    g = generator(seed)
    out = []
    for i in range(count):
        n = int(g.integers(n_range[0], n_range[1] + 1))
        kappa = float(10.0 ** g.uniform(*log10_kappa))
        nrhs = int(g.integers(nrhs_range[0], nrhs_range[1] + 1))
        out.append({"n": n, "kappa": kappa, "nrhs": nrhs, "seed": int(seed) * 100003 + i})
    return out


def batch_system_torch(spec: dict, device="cuda"):
    """One system of :func:`batch_specs` on ``device``: A from
    :func:`randsvd_problem_torch`, then ``nrhs`` solutions X ~ U(-1, 1) and
    B = A X in float64.  Returns (a, x_true, b) with x_true and b shaped
    (n, nrhs) as transposes of contiguous (nrhs, n) tensors."""
    import torch
    n, nrhs = spec["n"], spec["nrhs"]
    a, _, _ = randsvd_problem_torch(n, spec["kappa"], spec["seed"], device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(spec["seed"]) + 1)
    x = torch.rand((nrhs, n), generator=gen, dtype=torch.float64, device=device) * 2.0 - 1.0
    b = (x @ a.T).contiguous()
    return a, x.t(), b.t()
