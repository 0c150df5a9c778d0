"""Python binding of libgmresir (mixed-precision GMRES-IR with recycling).

Argument marshalling only: every step of the method runs in the HIP library
(``libgmresir.so``, C ABI in ``include/gmresir.h``).  PyTorch provides device
memory and the stream.  There is no fallback: when the library is missing or
cannot be loaded, every entry point raises.

Method: Oktay & Carson, "Mixed Precision GMRES-based Iterative Refinement
with Recycling" -- Algorithm 3 (RGMRES-IR), with GMRES-IR (Algorithm 2) as
the k = 0 case.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "GmresirError",
    "PREC",
    "STATUS",
    "library_path",
    "load_library",
    "default_opts",
    "factor",
    "import_factors",
    "Handle",
    "EXPORTED",
    "KERNEL_CLASSES",
    "timing_mask",
    "rank1",
    "solve_batched",
    "errors_noalloc",
    "TorchAllocator",
]

_HERE = os.path.dirname(os.path.abspath(__file__))

PREC = {"bf16": 1, "fp16": 2, "fp32": 3, "fp64": 4, "dd": 5}
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EINTERNAL",
          1: "ESINGULAR", 2: "ERANGE", 3: "ENOCONV"}
MAX_STEPS = 64
# kernel classes of gmresir_kernel_stats, bit 0 first
KERNEL_CLASSES = ("lu_panel", "lu_trsm", "lu_gemm", "trsv_lower", "trsv_upper", "gemv_au",
                  "residual", "ortho", "arnoldi_step", "arnoldi_cycle")


def timing_mask(classes, stride: int = 0) -> int:
    """opts.timing for the named kernel classes (bits 0-7 for classes 0-7,
    16-23 for classes 8-15) with every stride-th launch bracketed."""
    m = 0
    for c in classes:
        i = KERNEL_CLASSES.index(c)
        m |= 1 << (i if i < 8 else i + 8)
    return m | ((stride & 0xFF) << 8 if stride > 1 else 0)

# every symbol declared in include/gmresir.h
EXPORTED = (
    "gmresir_default_opts", "gmresir_factor", "gmresir_solve", "gmresir_free",
    "gmresir_strerror", "gmresir_last_error", "gmresir_import_factors",
    "gmresir_export_factors", "gmresir_apply", "gmresir_kernel_stats", "gmresir_query",
    "gmresir_solve_transposed", "gmresir_rank1", "gmresir_choose_k", "gmresir_solve_batched",
    "gmresir_errors", "gmresir_errors_noalloc",
)


class Opts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("uf", ctypes.c_int32),
        ("u", ctypes.c_int32),
        ("ur", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("imax", ctypes.c_int32),
        ("maxit", ctypes.c_int32),
        ("berr_target", ctypes.c_double),
        ("scale_pow2", ctypes.c_int32),
        ("keep_recycle", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("matvec_u", ctypes.c_int32),
        ("reuse_recycle", ctypes.c_int32),
        ("ortho", ctypes.c_int32),
        ("alloc", ctypes.c_void_p),
        ("free_", ctypes.c_void_p),
        ("alloc_user", ctypes.c_void_p),
    ]


class KernelStat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 24),
        ("launches", ctypes.c_int32),
        ("bound", ctypes.c_int32),
        ("total_ms", ctypes.c_double),
        ("work", ctypes.c_double),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("steps", ctypes.c_int32),
        ("total_its", ctypes.c_int32),
        ("its", ctypes.c_int32 * MAX_STEPS),
        ("berr", ctypes.c_double * (MAX_STEPS + 1)),
        ("singular_col", ctypes.c_int32),
        ("recycle_dim", ctypes.c_int32),
        ("t_factor_s", ctypes.c_double),
        ("t_solve_s", ctypes.c_double),
        ("berr_cw", ctypes.c_double * (MAX_STEPS + 1)),
        ("t_x0_s", ctypes.c_double),
        ("t_residual_s", ctypes.c_double),
        ("t_precond_s", ctypes.c_double),
        ("t_recycle_s", ctypes.c_double),
        ("t_arnoldi_s", ctypes.c_double),
        ("cycles_persistent", ctypes.c_int32),
        ("cycles_fallback", ctypes.c_int32),
    ]


class GmresirError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"gmresir status {status} ({STATUS.get(status, '?')}): {message}")
        self.status = status


class BatchItem(ctypes.Structure):
    _fields_ = [
        ("A", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("lda", ctypes.c_int64),
        ("b", ctypes.c_void_p),
        ("x", ctypes.c_void_p),
        ("nrhs", ctypes.c_int64),
        ("ldb", ctypes.c_int64),
        ("info", ctypes.c_void_p),
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


_LIB = None


def library_path() -> str:
    return os.environ.get("GMRESIR_LIB", os.path.join(_HERE, "libgmresir.so"))


def load_library() -> ctypes.CDLL:
    """Load libgmresir.so (raises OSError if it is missing)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise OSError(f"{path} not found: build it with `python -m paper_2201_09827_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.gmresir_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.gmresir_default_opts.restype = None
    lib.gmresir_factor.argtypes = [vp, i64, i64, ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
    lib.gmresir_factor.restype = ctypes.c_int
    lib.gmresir_solve.argtypes = [vp, vp, vp, i64, i64, vp, ctypes.POINTER(Info)]
    lib.gmresir_solve.restype = ctypes.c_int
    lib.gmresir_free.argtypes = [vp]
    lib.gmresir_free.restype = None
    lib.gmresir_strerror.argtypes = [ctypes.c_int]
    lib.gmresir_strerror.restype = ctypes.c_char_p
    lib.gmresir_last_error.argtypes = []
    lib.gmresir_last_error.restype = ctypes.c_char_p
    lib.gmresir_import_factors.argtypes = [vp, i64, i64, vp, i64, ctypes.POINTER(i32), i32,
                                           ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
    lib.gmresir_import_factors.restype = ctypes.c_int
    lib.gmresir_export_factors.argtypes = [vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.gmresir_export_factors.restype = ctypes.c_int
    lib.gmresir_apply.argtypes = [vp, i32, vp, vp, vp]
    lib.gmresir_apply.restype = ctypes.c_int
    lib.gmresir_errors.argtypes = [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.gmresir_errors.restype = ctypes.c_int
    lib.gmresir_errors_noalloc.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp]
    lib.gmresir_errors_noalloc.restype = ctypes.c_int
    lib.gmresir_kernel_stats.argtypes = [vp, ctypes.POINTER(KernelStat), i32, ctypes.POINTER(i32)]
    lib.gmresir_kernel_stats.restype = ctypes.c_int
    lib.gmresir_query.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    lib.gmresir_query.restype = ctypes.c_int
    lib.gmresir_solve_transposed.argtypes = [vp, vp, vp, i64, i64, vp, ctypes.POINTER(Info)]
    lib.gmresir_solve_transposed.restype = ctypes.c_int
    lib.gmresir_rank1.argtypes = [ctypes.c_double, vp, vp, i64, vp, i64, vp]
    lib.gmresir_rank1.restype = ctypes.c_int
    lib.gmresir_choose_k.argtypes = [vp, vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), vp]
    lib.gmresir_choose_k.restype = ctypes.c_int
    lib.gmresir_solve_batched.argtypes = [ctypes.POINTER(BatchItem), i64, ctypes.POINTER(Opts),
                                          i32, vp]
    lib.gmresir_solve_batched.restype = ctypes.c_int
    _LIB = lib
    return lib


def default_opts() -> Opts:
    o = Opts()
    load_library().gmresir_default_opts(ctypes.byref(o))
    return o


def _opts(**kw) -> Opts:
    o = default_opts()
    for key, val in kw.items():
        if key in ("uf", "u", "ur") and isinstance(val, str):
            val = PREC[val]
        if key == "ortho" and isinstance(val, str):
            val = {"cgs2": 0, "mgs": 1}[val]
        if key in ("keep_recycle", "scale_pow2", "timing", "matvec_u", "reuse_recycle"):
            val = int(val)
        if not hasattr(o, key):
            raise TypeError(f"unknown option {key!r}")
        setattr(o, key, val)
    return o


def _err(lib, status: int) -> GmresirError:
    msg = lib.gmresir_strerror(status).decode()
    last = lib.gmresir_last_error().decode()
    return GmresirError(status, f"{msg}; {last}" if last else msg)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_matrix(a):
    import torch
    if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64
            and a.dim() == 2 and a.shape[0] == a.shape[1] and a.stride(1) == 1):
        raise ValueError("A must be a square row-major float64 CUDA tensor")


def _info_dict(info: Info) -> dict:
    steps = int(info.steps)
    return {
        "status": int(info.status),
        "status_name": STATUS.get(int(info.status), "?"),
        "steps": steps,
        "total_its": int(info.total_its),
        "its": [int(info.its[i]) for i in range(min(steps, MAX_STEPS))],
        "berr": [float(info.berr[i]) for i in range(min(steps, MAX_STEPS) + 1)],
        "singular_col": int(info.singular_col),
        "recycle_dim": int(info.recycle_dim),
        "t_factor_s": float(info.t_factor_s),
        "t_solve_s": float(info.t_solve_s),
        "berr_cw": [float(info.berr_cw[i]) for i in range(min(steps, MAX_STEPS) + 1)],
        "t_x0_s": float(info.t_x0_s),
        "t_residual_s": float(info.t_residual_s),
        "t_precond_s": float(info.t_precond_s),
        "t_recycle_s": float(info.t_recycle_s),
        "t_arnoldi_s": float(info.t_arnoldi_s),
        "cycles_persistent": int(info.cycles_persistent),
        "cycles_fallback": int(info.cycles_fallback),
    }


class Handle:
    """A factorised matrix (owns the library handle)."""

    def __init__(self, lib, ptr: ctypes.c_void_p, n: int, opts: Opts, status: int):
        self._lib = lib
        self._ptr = ptr
        self.n = n
        self.opts = opts
        self.status = status

    def _live(self):
        if not self._ptr:
            raise RuntimeError("handle has been freed")
        return self._ptr

    def solve(self, b, stream=None):
        """Solve A x = b (b: float64 CUDA tensor, (n,) or (n, nrhs) column-major
        via the transpose of a C-contiguous (nrhs, n) tensor).  Returns
        (x, info) with info describing the last column; raises on a negative
        status, reports ENOCONV/ESINGULAR/ERANGE in info['status']."""
        return self._solve(self._lib.gmresir_solve, b, stream)

    def solve_transposed(self, g, stream=None):
        """Solve the adjoint system A^T lambda = g with the transposed factors
        and a recycle space of its own (same conventions as ``solve``)."""
        return self._solve(self._lib.gmresir_solve_transposed, g, stream)

    def choose_k(self, b, kmax: int, stream=None):
        """Automatic recycle dimension ("finding the knee"): one solve per
        k = 0 .. kmax; returns (k_best, its per k (-1: not converged or beyond
        the first-step limit), status)."""
        import torch
        ptr = self._live()
        if not (isinstance(b, torch.Tensor) and b.is_cuda and b.dtype == torch.float64
                and b.shape == (self.n,) and b.is_contiguous()):
            raise ValueError("b must be a contiguous float64 CUDA vector of length n")
        kb = ctypes.c_int32(0)
        its = (ctypes.c_int32 * (kmax + 1))()
        rc = self._lib.gmresir_choose_k(ptr, ctypes.c_void_p(b.data_ptr()), int(kmax),
                                        ctypes.byref(kb), its, _stream(stream))
        if rc < 0:
            raise _err(self._lib, rc)
        return int(kb.value), [int(v) for v in its], int(rc)

    def _solve(self, fn, b, stream):
        import torch
        ptr = self._live()
        if not (isinstance(b, torch.Tensor) and b.is_cuda and b.dtype == torch.float64):
            raise ValueError("b must be a float64 CUDA tensor")
        if b.dim() == 1:
            if b.shape[0] != self.n or b.stride(0) != 1:
                raise ValueError("b has the wrong length or stride")
            nrhs, ldb = 1, self.n
            x = torch.empty_like(b)
        else:
            bt = b.t()
            if b.shape[0] != self.n or not bt.is_contiguous():
                raise ValueError("2-D b must be the transpose of a contiguous (nrhs, n) tensor")
            nrhs, ldb = b.shape[1], self.n
            x = torch.empty((nrhs, self.n), dtype=torch.float64, device=b.device).t()
        info = Info()
        rc = fn(ptr, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), nrhs, ldb,
                _stream(stream), ctypes.byref(info))
        if rc < 0:
            raise _err(self._lib, rc)
        return x, _info_dict(info)

    def errors(self, b, x, x_true=None, stream=None):
        """Error measures of a solution from a double-double residual:
        returns (normwise backward error, componentwise backward error,
        forward error or nan without x_true)."""
        import torch
        ptr = self._live()
        for name, t in (("b", b), ("x", x), ("x_true", x_true)):
            if t is None and name == "x_true":
                continue
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                    and t.shape == (self.n,) and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 CUDA vector of length n")
        out = (ctypes.c_double * 3)()
        rc = self._lib.gmresir_errors(ptr, ctypes.c_void_p(b.data_ptr()),
                                      ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(x_true.data_ptr() if x_true is not None
                                                      else None),
                                      out, _stream(stream))
        if rc != 0:
            raise _err(self._lib, rc)
        return float(out[0]), float(out[1]), float(out[2])

    def apply(self, op: int, v, stream=None):
        """op 0: M^-1 v; op 1: A-tilde v; op 2: M^-T v; op 3: M^-T A_u^T v
        (all in u^2, returned in fp64)."""
        import torch
        ptr = self._live()
        if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.float64
                and v.shape == (self.n,) and v.is_contiguous()):
            raise ValueError("v must be a contiguous float64 CUDA vector of length n")
        y = torch.empty_like(v)
        rc = self._lib.gmresir_apply(ptr, int(op), ctypes.c_void_p(v.data_ptr()),
                                     ctypes.c_void_p(y.data_ptr()), _stream(stream))
        if rc != 0:
            raise _err(self._lib, rc)
        return y

    def export_factors(self):
        """(lu, ipiv, e): lu as numpy uint16 (fp16/bf16 bits) or float32,
        row-major n x n in logical (pivoted) row order; ipiv LAPACK style."""
        import numpy as np
        ptr = self._live()
        dt = np.float32 if self.opts.uf == PREC["fp32"] else np.uint16
        lu = np.empty((self.n, self.n), dtype=dt)
        ipiv = np.empty(self.n, dtype=np.int32)
        e = ctypes.c_int32(0)
        rc = self._lib.gmresir_export_factors(
            ptr, lu.ctypes.data_as(ctypes.c_void_p),
            ipiv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(e))
        if rc != 0:
            raise _err(self._lib, rc)
        return lu, ipiv, int(e.value)

    def kernel_stats(self) -> list:
        """Per-kernel-class launch timing (handle created with timing = a bit
        mask of KERNEL_CLASSES, 0xFF for all):
        list of dicts name, launches, bound ('hbm' or 'mfma'), total_ms, work
        (algorithmic bytes or flops summed over the launches)."""
        ptr = self._live()
        cap = 16
        arr = (KernelStat * cap)()
        cnt = ctypes.c_int32(0)
        rc = self._lib.gmresir_kernel_stats(ptr, arr, cap, ctypes.byref(cnt))
        if rc != 0:
            raise _err(self._lib, rc)
        return [{"name": arr[i].name.decode(), "launches": int(arr[i].launches),
                 "bound": "mfma" if arr[i].bound == 1 else "hbm",
                 "total_ms": float(arr[i].total_ms), "work": float(arr[i].work)}
                for i in range(cnt.value)]

    def free(self):
        if self._ptr:
            self._lib.gmresir_free(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


def factor(a, stream=None, **opts) -> Handle:
    """LU-factorise A (the factorisation step of Algorithm 3).  ``a``: square row-major float64
    CUDA tensor.  Options: uf, u, ur ('fp16', 'bf16', 'fp32', 'fp64', 'dd'),
    m, k, tau, imax, maxit, berr_target, scale_pow2, keep_recycle, timing,
    matvec_u, reuse_recycle, ortho ('cgs2' or 'mgs'), alloc / free_ (see
    TorchAllocator).  Raises
    GmresirError on a negative status; ESINGULAR/ERANGE return a handle whose
    ``status`` says so."""
    lib = load_library()
    _check_matrix(a)
    o = _opts(**opts)
    out = ctypes.c_void_p()
    rc = lib.gmresir_factor(ctypes.c_void_p(a.data_ptr()), a.shape[0], a.stride(0),
                            ctypes.byref(o), _stream(stream), ctypes.byref(out))
    if rc < 0:
        raise _err(lib, rc)
    return Handle(lib, out, a.shape[0], o, rc)


def import_factors(a, lu, ipiv, e: int, stream=None, **opts) -> Handle:
    """Handle from given factors: ``lu`` a CUDA tensor of u_f elements
    (int16/uint16 bits for fp16/bf16, float32 for fp32), row-major n x n in
    logical row order; ``ipiv`` a host sequence of n LAPACK-style 0-based
    interchanges; ``e`` the power-of-two scale."""
    import numpy as np
    lib = load_library()
    _check_matrix(a)
    o = _opts(**opts)
    piv = np.ascontiguousarray(np.asarray(ipiv, dtype=np.int32))
    out = ctypes.c_void_p()
    rc = lib.gmresir_import_factors(
        ctypes.c_void_p(a.data_ptr()), a.shape[0], a.stride(0), ctypes.c_void_p(lu.data_ptr()),
        lu.stride(0), piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(e),
        ctypes.byref(o), _stream(stream), ctypes.byref(out))
    if rc < 0:
        raise _err(lib, rc)
    return Handle(lib, out, a.shape[0], o, rc)


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class TorchAllocator:
    """The library's device buffers from torch's caching allocator (the
    opts.alloc / opts.free_ hooks): ``g.factor(A, **TorchAllocator().opts())``.
    Keep the object alive as long as handles created with it exist."""

    def __init__(self):
        import torch
        self.live = {}
        self.calls = 0

        def _alloc(nbytes, user):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes))
            except Exception:
                return None
            self.live[int(p)] = int(nbytes)
            self.calls += 1
            return int(p)

        def _free(ptr, user):
            if ptr is not None and int(ptr) in self.live:
                del self.live[int(ptr)]
                torch.cuda.caching_allocator_delete(int(ptr))

        self._alloc = _ALLOC_FN(_alloc)
        self._free = _FREE_FN(_free)

    def opts(self) -> dict:
        return {"alloc": ctypes.cast(self._alloc, ctypes.c_void_p).value,
                "free_": ctypes.cast(self._free, ctypes.c_void_p).value}


def errors_noalloc(a, b, x, out, x_true=None, stream=None) -> None:
    """gmresir_errors_noalloc: the three error measures of x written to the
    device tensor out (3 float64) in stream order, without a handle and
    without allocating (A: row-major float64 CUDA, 16-byte aligned, even
    leading dimension)."""
    import torch
    lib = load_library()
    _check_matrix(a)
    n = a.shape[0]
    for name, t in (("b", b), ("x", x), ("x_true", x_true)):
        if t is None and name == "x_true":
            continue
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.shape == (n,) and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float64 CUDA vector of length n")
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64
            and out.numel() >= 3 and out.is_contiguous()):
        raise ValueError("out must be a contiguous float64 CUDA tensor of 3 values")
    rc = lib.gmresir_errors_noalloc(ctypes.c_void_p(a.data_ptr()), n, a.stride(0),
                                    ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(x_true.data_ptr() if x_true is not None
                                                    else None),
                                    ctypes.c_void_p(out.data_ptr()), _stream(stream))
    if rc != 0:
        raise _err(lib, rc)


def rank1(alpha: float, x, y, out=None, stream=None):
    """out = alpha x y^T for float64 CUDA vectors x, y of length n (out: a new or
    given row-major n x n float64 CUDA tensor)."""
    import torch
    lib = load_library()
    n = x.shape[0]
    for v in (x, y):
        if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.float64
                and v.shape == (n,) and v.is_contiguous()):
            raise ValueError("x and y must be contiguous float64 CUDA vectors of one length")
    if out is None:
        out = torch.empty((n, n), dtype=torch.float64, device=x.device)
    _check_matrix(out)
    rc = lib.gmresir_rank1(float(alpha), ctypes.c_void_p(x.data_ptr()),
                           ctypes.c_void_p(y.data_ptr()), n, ctypes.c_void_p(out.data_ptr()),
                           out.stride(0), _stream(stream))
    if rc != 0:
        raise _err(lib, rc)
    return out


def solve_batched(systems, workers: int = 8, stream=None, **opts):
    """Factor and solve many independent systems (uneven n, each with its own
    right-hand sides) with the same options, several at once on worker
    streams.  ``systems``: sequence of (A, B) with A a square row-major float64
    CUDA tensor and B its right-hand sides, (n,) or the transpose of a
    contiguous (nrhs, n) tensor.  Returns a list of (X, infos, status) in the
    order given: X shaped like B, infos one dict per right-hand side, status
    the system's gmresir_status (ESINGULAR / ERANGE / ENOCONV are outcomes, not
    errors).  Raises GmresirError on a negative return."""
    import torch
    lib = load_library()
    o = _opts(**opts)
    items = (BatchItem * len(systems))()
    keep = []
    for i, (a, b) in enumerate(systems):
        _check_matrix(a)
        n = a.shape[0]
        if not (isinstance(b, torch.Tensor) and b.is_cuda and b.dtype == torch.float64):
            raise ValueError("b must be a float64 CUDA tensor")
        if b.dim() == 1:
            if b.shape[0] != n or b.stride(0) != 1:
                raise ValueError("b has the wrong length or stride")
            nrhs = 1
            x = torch.empty_like(b)
        else:
            if b.shape[0] != n or not b.t().is_contiguous():
                raise ValueError("2-D b must be the transpose of a contiguous (nrhs, n) tensor")
            nrhs = b.shape[1]
            x = torch.empty((nrhs, n), dtype=torch.float64, device=b.device).t()
        infos = (Info * nrhs)()
        keep.append((x, infos, nrhs))
        items[i] = BatchItem(a.data_ptr(), n, a.stride(0), b.data_ptr(), x.data_ptr(), nrhs, n,
                             ctypes.cast(infos, ctypes.c_void_p), 0, 0)
    rc = lib.gmresir_solve_batched(items, len(systems), ctypes.byref(o), int(workers),
                                   _stream(stream))
    if rc < 0:
        raise _err(lib, rc)
    return [(x, [_info_dict(infos[j]) for j in range(nrhs)], int(items[i].status))
            for i, (x, infos, nrhs) in enumerate(keep)]
