"""Helpers shared by the GPU parity tests (inputs, oracle runs, comparisons)."""
import sys

import numpy as np

from oracle import fp
from oracle.lu import fp16_scale_exponent, lu_blocked, unpack
from oracle.refine import Options

NB = 64  # block size of the library's LU (fixes its u_f rounding points)
U64 = 2.0 ** -53

_UF_NP = {"fp16": np.float16, "fp32": np.float32}


def log(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def oracle_options(uf="fp16", m=20, k=5, tau=1e-4, imax=10, maxit=0, berr=1e-14, u="fp32",
                   ur="fp64", matvec="u2", reuse=False, ortho="cgs2"):
    return Options(uf=uf, u=u, ur=ur, m=m, k=k, tau=tau, imax=imax, maxit=maxit,
                   berr_target=berr, nb=NB, matvec=matvec, reuse_recycle=reuse, ortho=ortho)


def lib_options(o: Options) -> dict:
    return dict(uf=o.uf, u=o.u, ur=o.ur, m=o.m, k=o.k, tau=o.tau, imax=o.imax,
                maxit=o.maxit, berr_target=o.berr_target,
                matvec_u=1 if o.matvec == "u" else 0, reuse_recycle=int(o.reuse_recycle),
                ortho=o.ortho)


def decode_factors(raw: np.ndarray, uf: str) -> np.ndarray:
    """u_f bits (uint16) or float32 from the library -> float64 values."""
    if uf == "fp16":
        return raw.view(np.float16).astype(np.float64)
    if uf == "bf16":
        return (raw.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return raw.astype(np.float64)


def encode_factors(lu: np.ndarray, uf: str) -> np.ndarray:
    """float64 array holding u_f values -> the library's storage bits."""
    if uf == "fp16":
        return lu.astype(np.float16).view(np.uint16)
    if uf == "bf16":
        b = lu.astype(np.float32).view(np.uint32)
        assert np.all((b & 0xFFFF) == 0)
        return (b >> 16).astype(np.uint16)
    return lu.astype(np.float32)


def oracle_factors(a: np.ndarray, uf: str):
    n = a.shape[0]
    e = fp16_scale_exponent(float(np.max(np.abs(a))), n) if uf == "fp16" else 0
    af = fp.fl(np.ldexp(a, e), uf)
    return lu_blocked(af, uf, NB), e, af


def ulp_distance(x: np.ndarray, y: np.ndarray, uf: str) -> np.ndarray:
    """Distance in units of the u_f spacing at max(|x|, |y|)."""
    fmt = fp.FORMATS[uf]
    m = np.maximum(np.abs(x), np.abs(y))
    _, ex = np.frexp(np.where(m > 0, m, 1.0))
    ex = np.maximum(ex - 1, fmt.emin)
    spacing = np.ldexp(1.0, ex - (fmt.p - 1))
    return np.abs(x - y) / spacing
