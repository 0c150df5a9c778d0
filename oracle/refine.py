"""Mixed-precision GMRES-IR with and without recycling (oracle driver).

Test infrastructure only.  Algorithm 3 of the paper (RGMRES-IR) with the
correction equation solved by :func:`oracle.krylov.gcrodr`; k = 0 gives
Algorithm 2 (GMRES-IR with restarted GMRES(m)).

Build-mode readings (the paper leaves these open):

* A, b and x are held in float64 whatever u is; the inner solver works in u.
  (Storing x in u would cap the attainable backward error at u.)
* A_u = fl_u(A) is the matrix used by the preconditioned product; with u =
  fp64 it is A itself.
* Factorisation: A_f = fl_uf(2^e A) with the power-of-two scale of
  :func:`oracle.lu.fp16_scale_exponent` for fp16 (e = 0 otherwise), then
  blocked GEPP (:func:`oracle.lu.lu_blocked`).  M = 2^-e P^T L U.
* The preconditioned operator is A-tilde = U^-1 L^-1 P A (the paper omits P)
  scaled by 2^e; A-tilde v is computed in u^2 (fp64 for u = fp32,
  double-double for u = fp64) with A_u, L and U taken exactly, and the single
  result rounded to u.  The preconditioned right-hand side M^-1 r-hat uses
  the same triangular solves.
* x0 = M^-1 b computed with the same u^2 triangular solves, kept in fp64
  (the paper substitutes in u_f).
* Refinement step i: r = b - A x in u_r (fp64, or double-double rounded to
  fp64); eta = ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf); stop when
  eta <= berr_target; otherwise s = ||r||_inf, r-hat = fl_u(r / s),
  z = fl_u(M^-1 r-hat), d = GCRO-DR(z), x = x + s d (fp64).
  After i_max corrections the final residual is evaluated once more.
* Status: 0 converged, 1 exact zero pivot, 2 non-finite data or overflow in
  u_f, 3 not converged within i_max.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import fp
from .fp import fl
from .krylov import KrylovOptions, RecycleState, gcrodr
from .lu import fp16_scale_exponent, lu_blocked, lu_chop, unpack

__all__ = ["Options", "Factors", "Info", "factor", "solve", "gmresir",
           "minv_t", "atilde_t", "residual_t", "solve_transposed", "gradient", "choose_k",
           "STATUS_OK", "STATUS_SINGULAR", "STATUS_RANGE", "STATUS_NOCONV"]

STATUS_OK = 0
STATUS_SINGULAR = 1
STATUS_RANGE = 2
STATUS_NOCONV = 3

_ORDER = {"fp16": 0, "bf16": 0, "fp32": 1, "fp64": 2, "dd": 3}


@dataclass
class Options:
    uf: str = "fp16"
    u: str = "fp32"
    ur: str = "fp64"
    m: int = 20
    k: int = 0
    tau: float = 1e-4
    imax: int = 10
    maxit: int = 0            # per correction solve; 0 -> 10 m
    berr_target: float = 1e-14
    nb: int = 64              # LU block size (rounding points depend on it)
    scale_pow2: bool | None = None   # None -> on for fp16 only
    ortho: str = "cgs2"
    keep_recycle: bool = False
    mode: str = "build"       # "build" or "paper" (chop-style LU, x in u)
    matvec: str = "u2"        # "u2": A-tilde v in u^2 (Algorithms 2, 3); "u": uniform u
    reuse_recycle: bool = False  # keep (U_k, C_k) between refinement steps

    def validate(self):
        if self.uf not in ("fp16", "bf16", "fp32", "fp64"):
            raise ValueError("uf")
        if self.u not in ("fp32", "fp64"):
            raise ValueError("u")
        if self.ur not in ("fp64", "dd"):
            raise ValueError("ur")
        if not (_ORDER[self.uf] <= _ORDER[self.u] <= _ORDER[self.ur]):
            raise ValueError("precisions must satisfy uf >= u >= ur")
        if self.k < 0 or self.m <= self.k or self.m < 1:
            raise ValueError("need m > k >= 0")
        if not (self.tau > 0):
            raise ValueError("tau")
        if self.matvec not in ("u2", "u"):
            raise ValueError("matvec")
        if self.matvec == "u" and self.u != "fp64":
            raise ValueError("uniform-precision products are defined for u = fp64")

    def scaled(self) -> bool:
        return (self.uf == "fp16") if self.scale_pow2 is None else bool(self.scale_pow2)


@dataclass
class Factors:
    n: int
    opts: Options
    a: np.ndarray          # fp64
    au: np.ndarray         # u values (float64 array)
    lu: np.ndarray         # packed factors, u_f values
    ipiv: np.ndarray
    perm: np.ndarray
    e: int                 # scale exponent
    norm_a_inf: float
    L: np.ndarray
    U: np.ndarray
    status: int = 0
    info: int = 0


@dataclass
class Info:
    status: int = 0
    steps: int = 0
    its: list = field(default_factory=list)      # Arnoldi steps per correction
    berr: list = field(default_factory=list)     # eta_N per refinement step
    cycles: list = field(default_factory=list)
    resid_log: list = field(default_factory=list)

    @property
    def total_its(self) -> int:
        return int(sum(self.its))

    def paper_format(self) -> str:
        return f"{self.total_its} ({','.join(str(i) for i in self.its)})"


def factor(a: np.ndarray, opts: Options) -> Factors:
    """The factorisation step of Algorithm 3: LU in u_f (with conversions)."""
    opts.validate()
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    n = a.shape[0]
    if not np.all(np.isfinite(a)):
        f = Factors(n, opts, a, a, a, np.arange(n), np.arange(n), 0, math.inf,
                    a, a, STATUS_RANGE, 0)
        return f
    au = fl(a, opts.u)
    e = fp16_scale_exponent(float(np.max(np.abs(a))), n) if opts.scaled() else 0
    af = fl(np.ldexp(a, e), opts.uf)
    if opts.mode == "paper":
        res = lu_chop(af, opts.uf)
    else:
        res = lu_blocked(af, opts.uf, opts.nb)
    L, U = unpack(res.lu)
    status = STATUS_OK
    if res.info:
        status = STATUS_SINGULAR
    elif not np.all(np.isfinite(res.lu)) or not np.all(np.isfinite(af)):
        status = STATUS_RANGE
    norm_a = float(np.max(np.sum(np.abs(a), axis=1)))
    return Factors(n, opts, a, au, res.lu, res.ipiv, res.perm, e, norm_a, L, U,
                   status, res.info)


# ---------------------------------------------------------------------------
# preconditioned products in u^2
# ---------------------------------------------------------------------------

def _dd_lower_unit(L, th, tl):
    n = L.shape[0]
    yh, yl = th.copy(), tl.copy()
    for j in range(n - 1):
        col = L[j + 1:, j]
        p, e = fp.two_prod(col, yh[j])
        e = e + col * yl[j]
        yh[j + 1:], yl[j + 1:] = fp.dd_add(yh[j + 1:], yl[j + 1:], -p, -e)
    return yh, yl


def _dd_upper(U, th, tl):
    n = U.shape[0]
    yh, yl = th.copy(), tl.copy()
    for j in range(n - 1, -1, -1):
        qh, ql = fp.dd_div_d(yh[j], yl[j], U[j, j])
        yh[j], yl[j] = qh, ql
        if j > 0:
            col = U[:j, j]
            p, e = fp.two_prod(col, qh)
            e = e + col * ql
            yh[:j], yl[:j] = fp.dd_add(yh[:j], yl[:j], -p, -e)
    return yh, yl


def minv_hi(f: Factors, v: np.ndarray, wide: str):
    """M^-1 v = 2^e U^-1 L^-1 P v in precision ``wide`` (fp64 or dd);
    returns the float64 (rounded) result."""
    if wide == "fp64":
        t = v[f.perm]
        y = sla.solve_triangular(f.L, t, lower=True, unit_diagonal=True,
                                 check_finite=False)
        z = sla.solve_triangular(f.U, y, lower=False, check_finite=False)
        return np.ldexp(z, f.e)
    th = np.array(v, dtype=np.float64)[f.perm]
    tl = np.zeros_like(th)
    yh, yl = _dd_lower_unit(f.L, th, tl)
    zh, zl = _dd_upper(f.U, yh, yl)
    return np.ldexp(zh + zl, f.e)


def atilde(f: Factors, v: np.ndarray) -> np.ndarray:
    """fl_u(A-tilde v) with all arithmetic in u^2 (Algorithms 2 and 3)."""
    u = f.opts.u
    wide = fp.square_precision(u)
    if wide == "fp64":
        w = f.au @ v
        return fl(minv_hi(f, w, "fp64"), u)
    # u = fp64: double-double product, then double-double solves
    wh, wl = fp.dd_gemv(f.au, v)
    wh = wh[f.perm]
    wl = wl[f.perm]
    yh, yl = _dd_lower_unit(f.L, wh, wl)
    zh, zl = _dd_upper(f.U, yh, yl)
    return np.ldexp(zh + zl, f.e)


def atilde64(f: Factors, y: np.ndarray) -> np.ndarray:
    """A-tilde Y for a float64 block (recycle set-up), rounded to fp64."""
    wide = fp.square_precision(f.opts.u)
    out = np.zeros_like(y)
    for c in range(y.shape[1]):
        if wide == "fp64":
            out[:, c] = minv_hi(f, f.au @ y[:, c], "fp64")
        else:
            wh, wl = fp.dd_gemv(f.au, y[:, c])
            yh, yl = _dd_lower_unit(f.L, wh[f.perm], wl[f.perm])
            zh, zl = _dd_upper(f.U, yh, yl)
            out[:, c] = np.ldexp(zh + zl, f.e)
    return out


def residual(f: Factors, b: np.ndarray, x: np.ndarray) -> np.ndarray:
    """r = b - A x in u_r, rounded to fp64."""
    if f.opts.ur == "fp64":
        return b - f.a @ x
    rh, rl = fp.dd_gemv(f.a, x, y0h=b, y0l=np.zeros_like(b), sign=-1.0)
    return rh + rl


def backward_error(f: Factors, b, x, r, norm_a: float | None = None) -> float:
    na = f.norm_a_inf if norm_a is None else norm_a
    den = na * float(np.max(np.abs(x))) + float(np.max(np.abs(b)))
    num = float(np.max(np.abs(r)))
    if num == 0.0:
        return 0.0
    return num / den if den > 0 else math.inf


# ---------------------------------------------------------------------------
# Algorithm 3
# ---------------------------------------------------------------------------

# ---------------------------------------------------------------------------
# the adjoint system A^T lambda = g with the same factors:
# P 2^e A = L U gives A^T = 2^-e U^T L^T P, so M^-T = 2^e P^T L^-T U^-T
# ---------------------------------------------------------------------------

def minv_t(f: Factors, v: np.ndarray) -> np.ndarray:
    """M^-T v = 2^e P^T L^-T U^-T v in fp64 ((P^T z)[perm[i]] = z[i])."""
    y = sla.solve_triangular(f.U, v, lower=False, trans="T", check_finite=False)
    z = sla.solve_triangular(f.L, y, lower=True, unit_diagonal=True, trans="T",
                             check_finite=False)
    out = np.empty_like(z)
    out[f.perm] = z
    return np.ldexp(out, f.e)


def atilde_t(f: Factors, v: np.ndarray) -> np.ndarray:
    """fl_u(M^-T A_u^T v) with the arithmetic in u^2 = fp64 (u = fp32)."""
    return fl(minv_t(f, f.au.T @ v), f.opts.u)


def atilde64_t(f: Factors, y: np.ndarray) -> np.ndarray:
    out = np.zeros_like(y)
    for c in range(y.shape[1]):
        out[:, c] = minv_t(f, f.au.T @ y[:, c])
    return out


def residual_t(f: Factors, g: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """g - A^T lambda in fp64."""
    return g - f.a.T @ lam


def solve_transposed(f: Factors, g: np.ndarray, state: RecycleState | None = None):
    """The refinement loop of Algorithm 3 applied to A^T lambda = g with the
    transposed factors (u = fp32, u_r = fp64); ||A^T||_inf = ||A||_1.
    Returns (lambda, Info)."""
    o = f.opts
    if o.u != "fp32" or o.ur != "fp64" or o.mode != "build":
        raise ValueError("the adjoint solve is defined for u = fp32, u_r = fp64, build mode")
    norm_a1 = float(np.max(np.sum(np.abs(f.a), axis=0)))
    return _refine(f, g, state, None,
                   lambda v: minv_t(f, v), lambda v: atilde_t(f, v),
                   lambda y: atilde64_t(f, y), lambda bb, x: residual_t(f, bb, x), norm_a1)


def gradient(f: Factors, x: np.ndarray, gx: np.ndarray, state: RecycleState | None = None):
    """Gradient of a loss through x = A^-1 b: with g = dL/dx the adjoint
    lambda = A^-T g gives dL/db = lambda and dL/dA = -lambda x^T.
    Returns (dA, db, Info of the adjoint solve)."""
    lam, info = solve_transposed(f, gx, state)
    return -np.outer(lam, x), lam, info


def atilde_uniform(f: Factors, v: np.ndarray) -> np.ndarray:
    """A-tilde v with every operation in the working precision u = fp64
    (SGMRES-IR / RSGMRES-IR: uniform precision within GMRES, Section 3)."""
    return minv_hi(f, f.au @ v, "fp64")


def solve(f: Factors, b: np.ndarray, state: RecycleState | None = None,
          x0: np.ndarray | None = None):
    """Refinement loop of Algorithm 3 (k = 0: Algorithm 2).  Returns (x, Info).
    With matvec = "u" the correction solve applies M^-1 (to r-hat and inside
    GMRES) in u instead of u^2; x0 keeps u^2."""
    wide = fp.square_precision(f.opts.u)
    if f.opts.matvec == "u":
        return _refine(f, b, state, x0,
                       lambda v: minv_hi(f, v, wide), lambda v: atilde_uniform(f, v),
                       lambda y: np.column_stack([atilde_uniform(f, y[:, c])
                                                  for c in range(y.shape[1])]),
                       lambda bb, x: residual(f, bb, x), None,
                       minv_z=lambda v: minv_hi(f, v, "fp64"))
    return _refine(f, b, state, x0,
                   lambda v: minv_hi(f, v, wide), lambda v: atilde(f, v),
                   lambda y: atilde64(f, y), lambda bb, x: residual(f, bb, x), None)


def _refine(f: Factors, b: np.ndarray, state, x0, minv, apply_u, apply64, resid, norm_a,
            minv_z=None):
    o = f.opts
    minv_z = minv if minv_z is None else minv_z
    info = Info()
    if f.status != STATUS_OK:
        info.status = f.status
        return np.zeros(f.n), info
    b = np.asarray(b, dtype=np.float64)
    if not np.all(np.isfinite(b)):
        info.status = STATUS_RANGE
        return np.zeros(f.n), info
    if state is None or not o.keep_recycle:
        state = RecycleState()
    if x0 is not None:
        x = np.array(x0, dtype=np.float64)
    elif o.mode == "paper":
        # substitution in u_f, stored in u (the paper's initial solve)
        t = b[f.perm]
        y = np.zeros(f.n)
        for i in range(f.n):
            y[i] = fl(t[i] - fl(f.L[i, :i] @ y[:i], o.uf), o.uf)
        x = np.zeros(f.n)
        for i in range(f.n - 1, -1, -1):
            x[i] = fl((y[i] - fl(f.U[i, i + 1:] @ x[i + 1:], o.uf)) / f.U[i, i], o.uf)
        x = fl(np.ldexp(x, f.e), o.u)
    else:
        x = minv(b)
    kopts = KrylovOptions(m=o.m, k=o.k, tau=o.tau, maxit=o.maxit, u=o.u,
                          ortho=o.ortho, reuse=o.reuse_recycle)
    for i in range(o.imax + 1):
        r = resid(b, x)
        eta = backward_error(f, b, x, r, norm_a)
        info.berr.append(eta)
        if eta <= o.berr_target:
            info.steps = i
            info.status = STATUS_OK
            return x, info
        if i == o.imax:
            break
        s = float(np.max(np.abs(r)))
        rhat = fl(r / s, o.u)
        z = fl(minv_z(rhat), o.u)
        d, rec = gcrodr(apply_u, apply64, z, kopts, state, info.resid_log)
        info.its.append(rec.its)
        info.cycles.append(rec.cycles)
        if o.mode == "paper":
            x = fl(x + fl(s * d, o.u), o.u)
        else:
            x = x + s * d
    info.steps = o.imax
    info.status = STATUS_NOCONV
    return x, info


def gmresir(a: np.ndarray, b: np.ndarray, opts: Options):
    """Factor and solve in one call; returns (x, Info, Factors)."""
    f = factor(a, opts)
    x, info = solve(f, b)
    return x, info, f


def choose_k(f: Factors, b: np.ndarray, kmax: int):
    """Automatic recycle dimension, "finding the knee" (Section 3, total
    iterations against k): one solve per k = 0 .. kmax with the same factors
    and no recycle space carried between them; the chosen k is the smallest
    with the fewest total Arnoldi steps among the converged solves, limited to
    k <= (Arnoldi steps of the first refinement step at k = 0) - 1.
    Returns (k_best, its per k with -1 for not converged / beyond the limit)."""
    import dataclasses
    its = []
    best, best_its = 0, None
    limit = kmax
    for k in range(kmax + 1):
        if k > limit:
            its.append(-1)
            continue
        fk = dataclasses.replace(f, opts=dataclasses.replace(f.opts, k=k, keep_recycle=False))
        _, info = solve(fk, b)
        total = info.total_its if info.status == STATUS_OK else -1
        its.append(total)
        if k == 0:
            limit = max(0, info.its[0] - 1) if info.steps > 0 else 0
        if total >= 0 and (best_its is None or total < best_its):
            best, best_its = k, total
    return best, its

