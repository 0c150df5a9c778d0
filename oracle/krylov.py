"""GMRES(m) and GCRO-DR(m, k) for the correction equation (oracle).

Test infrastructure only.  Follows Algorithm "GCRO-DR" in Section 2 of the
paper (Parks et al. 2006) as used inside RGMRES-IR (Algorithm 3), on a
preconditioned operator passed as a callback.  With k = 0 every cycle is a
plain GMRES(m) cycle, which is GMRES-IR's correction solve (Algorithm 2);
the paper compares RGMRES-IR(m, k) against GMRES-IR with the same m
(Section 3).

Readings of the paper used here (the paper is silent or has misprints):

* initial guess d0 = 0; convergence when the residual estimate of the
  Givens-rotated least-squares problem drops to tau * ||z||_2 (relative
  preconditioned residual, Section 4);
* Arnoldi vectors and the iterate are stored in the working precision u;
  inner products, norms and linear combinations are formed in float64 and the
  stored vector is rounded to u once per operation; Hessenberg entries and
  all small dense problems are float64;
* the recycle pair (U_k, C_k) is stored in float64 and its QR factorisation
  is done in float64;
* orthogonalisation against [C_k, V_j] is classical Gram-Schmidt applied
  twice (CGS2) by default, or modified Gram-Schmidt (MGS);
* v_1 = r / ||r||_2 (the algorithm prints ||r||^2), the harmonic Ritz
  vectors of a later cycle use V-hat (printed v_m) and C_k = W-hat Q
  (printed W_{m+1}); D_k = diag(1 / ||U_k e_i||_2);
* the least-squares right-hand side W-hat^T r is taken as [C_k^T r; beta e1]
  with C_k^T r formed explicitly, so the first k rows are solved exactly by
  y1 = D^-1 (C_k^T r - B y2) and y2 solves the Hessenberg problem;
* W-hat^T V-hat uses C_k^T V = 0 and V_{j+1}^T V_j = [I; 0] by
  construction; C_k^T U-tilde and V_{j+1}^T U-tilde are formed;
* the k harmonic Ritz vectors belong to the k smallest |theta| (infinite
  values last); a complex pair contributes its real and imaginary parts and
  is dropped whole if it does not fit, so the dimension may become k - 1;
* a cycle that stops early (fewer steps than available) still refreshes the
  recycle space from its j steps; with j = 0 nothing is refreshed;
* "GMRES iterations" count Arnoldi steps only; the total per correction
  solve is capped by ``maxit`` (then the current iterate is returned).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .fp import fl

__all__ = [
    "KrylovOptions",
    "RecycleState",
    "CycleRecord",
    "SolveRecord",
    "givens_lsq",
    "harmonic_ritz_first",
    "harmonic_ritz_general",
    "select_ritz",
    "qr_positive",
    "gcrodr",
]


@dataclass
class KrylovOptions:
    m: int = 20
    k: int = 0
    tau: float = 1e-4
    maxit: int = 0          # 0 -> 10 * m
    u: str = "fp32"         # storage precision of Krylov vectors and d, r
    ortho: str = "cgs2"     # "cgs2" or "mgs"
    reuse: bool = False     # keep (U_k, C_k) of the previous solve (same A) as they are

    def cap(self) -> int:
        return self.maxit if self.maxit > 0 else 10 * self.m


@dataclass
class RecycleState:
    """U_k carried between correction solves (Ytilde_k = U_k, Alg. GCRO-DR
    last line), and C_k with it: at the end of every cycle A-tilde U_k = C_k
    with C_k orthonormal, so for an unchanged matrix the pair can be kept
    instead of recomputing QR(A-tilde U_k) (the reuse variant)."""
    U: np.ndarray | None = None
    C: np.ndarray | None = None

    @property
    def dim(self) -> int:
        return 0 if self.U is None else self.U.shape[1]


@dataclass
class CycleRecord:
    steps: int
    kind: str                 # "gmres" or "gcrodr"
    resid_est: float
    recycle_dim: int


@dataclass
class SolveRecord:
    its: int = 0
    cycles: list = field(default_factory=list)
    converged: bool = False
    final_resid: float = 0.0
    beta0: float = 0.0


def qr_positive(z: np.ndarray):
    """Reduced Householder QR with a positive diagonal of R."""
    q, r = np.linalg.qr(z)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :], r * s[:, None]


# ---------------------------------------------------------------------------
# Givens least squares (the min ||c - H y|| of GMRES)
# ---------------------------------------------------------------------------

class _Givens:
    """Progressive Givens QR of the (j+1) x j Hessenberg matrix."""

    def __init__(self, beta: float, size: int):
        self.cs = np.zeros(size)
        self.sn = np.zeros(size)
        self.g = np.zeros(size + 1)
        self.g[0] = beta
        self.R = np.zeros((size + 1, size))

    def add_column(self, j: int, h: np.ndarray) -> float:
        """Rotate column j (length j+2) and return the residual estimate."""
        h = np.array(h, dtype=np.float64)
        for i in range(j):
            t = self.cs[i] * h[i] + self.sn[i] * h[i + 1]
            h[i + 1] = -self.sn[i] * h[i] + self.cs[i] * h[i + 1]
            h[i] = t
        a, b = h[j], h[j + 1]
        rr = float(np.hypot(a, b))
        if rr == 0.0:
            c, s = 1.0, 0.0
        else:
            c, s = a / rr, b / rr
        self.cs[j], self.sn[j] = c, s
        h[j] = c * a + s * b
        h[j + 1] = 0.0
        self.g[j + 1] = -s * self.g[j]
        self.g[j] = c * self.g[j]
        self.R[: j + 2, j] = h
        return abs(self.g[j + 1])

    def solve(self, j: int) -> np.ndarray:
        if j == 0:
            return np.zeros(0)
        return sla.solve_triangular(self.R[:j, :j], self.g[:j], lower=False)


def givens_lsq(hbar: np.ndarray, beta: float):
    """y minimising ||beta e1 - Hbar y||_2 by Givens rotations and the
    resulting residual norm (used to pin the rotations against lstsq)."""
    j = hbar.shape[1]
    gv = _Givens(beta, j)
    est = beta
    for c in range(j):
        est = gv.add_column(c, hbar[: c + 2, c])
    return gv.solve(j), est


# ---------------------------------------------------------------------------
# harmonic Ritz vectors
# ---------------------------------------------------------------------------

def select_ritz(theta: np.ndarray, vecs: np.ndarray, k: int) -> np.ndarray:
    """Real basis of the eigenvectors of the k smallest |theta|.

    Infinite or NaN theta sort last; ties keep the solver's order.  A complex
    eigenvalue contributes Re z and Im z of one member of its conjugate pair;
    if both do not fit, selection stops (the dimension may be k - 1)."""
    theta = np.asarray(theta)
    mag = np.abs(theta)
    mag = np.where(np.isfinite(mag), mag, np.inf)
    order = np.argsort(mag, kind="stable")
    cols = []
    used = np.zeros(theta.size, dtype=bool)
    for idx in order:
        if len(cols) >= k:
            break
        if used[idx]:
            continue
        th = theta[idx]
        z = vecs[:, idx]
        if np.iscomplexobj(theta) and np.isfinite(th) and th.imag != 0.0:
            if len(cols) + 2 > k:
                break
            # mark the conjugate partner
            cand = np.where(~used)[0]
            cand = cand[cand != idx]
            if cand.size:
                partner = cand[np.argmin(np.abs(theta[cand] - np.conj(th)))]
                used[partner] = True
            used[idx] = True
            cols.append(np.real(z))
            cols.append(np.imag(z))
        else:
            used[idx] = True
            cols.append(np.real(z))
    if not cols:
        return np.zeros((vecs.shape[0], 0))
    return np.column_stack(cols).astype(np.float64)


def harmonic_ritz_first(hbar: np.ndarray, k: int) -> np.ndarray:
    """First-cycle harmonic Ritz vectors (Alg. GCRO-DR, GMRES branch):
    eigenvectors of H_j + h_{j+1,j}^2 H_j^{-T} e_j e_j^T."""
    j = hbar.shape[1]
    hm = hbar[:j, :j]
    hlast = hbar[j, j - 1]
    ej = np.zeros(j)
    ej[-1] = 1.0
    f = np.linalg.solve(hm.T, ej)
    mat = hm.copy()
    mat[:, -1] += hlast * hlast * f
    theta, vecs = np.linalg.eig(mat)
    return select_ritz(theta, vecs, k)


def harmonic_ritz_general(gbar: np.ndarray, wtv: np.ndarray, k: int) -> np.ndarray:
    """Later-cycle harmonic Ritz vectors (Alg. GCRO-DR, loop body):
    G^T G z = theta G^T (W^T V) z, solved by the QZ algorithm."""
    lhs = gbar.T @ gbar
    rhs = gbar.T @ wtv
    theta, vecs = sla.eig(lhs, rhs)
    return select_ritz(theta, vecs, k)


# ---------------------------------------------------------------------------
# Arnoldi on (I - C C^T) A
# ---------------------------------------------------------------------------

def _orthogonalise(w, basis, u, scheme):
    """Return (w_orth, coefficients) for w against the columns of ``basis``."""
    if basis.shape[1] == 0:
        return w, np.zeros(0)
    if scheme == "cgs2":
        h1 = basis.T @ w
        w = fl(w - basis @ h1, u)
        h2 = basis.T @ w
        w = fl(w - basis @ h2, u)
        return w, h1 + h2
    if scheme == "mgs":
        h = np.zeros(basis.shape[1])
        for i in range(basis.shape[1]):
            h[i] = basis[:, i] @ w
            w = fl(w - h[i] * basis[:, i], u)
        return w, h
    raise ValueError(scheme)


def _arnoldi(apply_u, r, C, nsteps, tol, opts, record_resid=None):
    """Up to ``nsteps`` Arnoldi steps from v1 = r/||r|| with the projected
    operator (I - C C^T) A.  Stops early when the Givens estimate <= tol or
    on exact breakdown.  Returns V (n x (j+1)), Hbar, B, j, Givens, beta."""
    u = opts.u
    n = r.size
    kc = 0 if C is None else C.shape[1]
    beta = float(np.linalg.norm(r))
    V = np.zeros((n, nsteps + 1))
    V[:, 0] = fl(r / beta, u)
    H = np.zeros((nsteps + 1, nsteps))
    B = np.zeros((kc, nsteps))
    gv = _Givens(beta, nsteps)
    j = 0
    est = beta
    while j < nsteps:
        w = apply_u(V[:, j])
        basis = V[:, : j + 1] if kc == 0 else np.hstack([C, V[:, : j + 1]])
        w, h = _orthogonalise(w, basis, u, opts.ortho)
        B[:, j] = h[:kc]
        H[: j + 1, j] = h[kc:]
        hn = float(np.linalg.norm(w))
        H[j + 1, j] = hn
        est = gv.add_column(j, H[: j + 2, j])
        if record_resid is not None:
            record_resid.append(est)
        if hn > 0.0:
            V[:, j + 1] = fl(w / hn, u)
        j += 1
        if hn == 0.0 or est <= tol:
            break
    return V[:, : j + 1], H[: j + 1, :j], B[:, :j], j, gv, beta, est


def gcrodr(apply_u, apply64, z, opts: KrylovOptions, state: RecycleState,
           resid_log: list | None = None):
    """Solve A-tilde d = z with d0 = 0 by GCRO-DR(m, k) (k = 0: GMRES(m)).

    ``apply_u(v)``: fl_u(A-tilde v) for a vector of u values;
    ``apply64(Y)``: A-tilde Y in float64 for an n x c float64 block.
    ``state`` holds U_k on entry (or None) and receives the new U_k.
    Returns (d, SolveRecord); d holds u values.
    """
    u = opts.u
    m, k = opts.m, opts.k
    cap = opts.cap()
    n = z.size
    rec = SolveRecord()
    beta0 = float(np.linalg.norm(z))
    rec.beta0 = beta0
    d = np.zeros(n)
    r = np.array(z, dtype=np.float64)
    if beta0 == 0.0:
        rec.converged = True
        return d, rec
    tol = opts.tau * beta0
    C = U = None

    # --- a recycled space from the previous system: QR of A-tilde Ytilde
    if k > 0 and state.U is not None and state.U.shape[1] > 0:
        if opts.reuse and state.C is not None:
            C, U = state.C, state.U
        else:
            yt = state.U
            zq = apply64(yt)
            q, rr = qr_positive(zq)
            C = q
            U = sla.solve_triangular(rr, yt.T, lower=False, trans="T").T  # Yt R^-1
        c = C.T @ r
        d = fl(U @ c, u)
        r = fl(r - C @ c, u)

    while True:
        rn = float(np.linalg.norm(r))
        rec.final_resid = rn
        if rn <= tol:
            rec.converged = True
            break
        if rec.its >= cap:
            break
        kc = 0 if C is None else C.shape[1]
        nsteps = min(m - kc, cap - rec.its)
        if kc == 0:
            # plain GMRES cycle (first cycle of GCRO-DR, or GMRES(m))
            V, Hb, _, j, gv, beta, est = _arnoldi(apply_u, r, None, nsteps, tol,
                                                   opts, resid_log)
            y = gv.solve(j)
            d = fl(d + V[:, :j] @ y, u)
            r = fl(r - V[:, : j + 1] @ (Hb @ y), u)
            rec.its += j
            rec.cycles.append(CycleRecord(j, "gmres", est, 0))
            if k > 0 and j > 0:
                pk = harmonic_ritz_first(Hb, k)
                if pk.shape[1] > 0:
                    ytil = V[:, :j] @ pk
                    q, rr = qr_positive(Hb @ pk)
                    C = V[:, : j + 1] @ q
                    U = sla.solve_triangular(rr, ytil.T, lower=False, trans="T").T
        else:
            ctr = C.T @ r
            V, Hb, B, j, gv, beta, est = _arnoldi(apply_u, r, C, nsteps, tol,
                                                   opts, resid_log)
            y2 = gv.solve(j)
            dk = 1.0 / np.linalg.norm(U, axis=0)
            ut = U * dk[None, :]
            y1 = (ctr - B @ y2) / dk
            d = fl(d + ut @ y1 + V[:, :j] @ y2, u)
            r = fl(r - C @ (dk * y1 + B @ y2) - V[:, : j + 1] @ (Hb @ y2), u)
            rec.its += j
            rec.cycles.append(CycleRecord(j, "gcrodr", est, kc))
            if j > 0:
                gbar = np.zeros((kc + j + 1, kc + j))
                gbar[:kc, :kc] = np.diag(dk)
                gbar[:kc, kc:] = B
                gbar[kc:, kc:] = Hb
                wtv = np.zeros((kc + j + 1, kc + j))
                wtv[:kc, :kc] = C.T @ ut
                wtv[kc:, :kc] = V[:, : j + 1].T @ ut
                wtv[kc:, kc:] = np.eye(j + 1, j)
                pk = harmonic_ritz_general(gbar, wtv, k)
                if pk.shape[1] > 0:
                    vhat = np.hstack([ut, V[:, :j]])
                    what = np.hstack([C, V[:, : j + 1]])
                    ytil = vhat @ pk
                    q, rr = qr_positive(gbar @ pk)
                    C = what @ q
                    U = sla.solve_triangular(rr, ytil.T, lower=False, trans="T").T
    if k > 0:
        state.U = None if U is None else U.copy()
        state.C = None if C is None else C.copy()
    return d, rec
