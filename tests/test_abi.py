"""The C-ABI library loads and exports every symbol include/gmresir.h
declares; the ctypes structures match the C layout (checked against a probe
compiled from the header with gcc).  No compute call is made (no GPU here)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

import paper_2201_09827_amd as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmresir.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(gmresir_[a-z0-9_]+)\s*\(", text)))


def test_header_declarations_match_binding_list():
    assert _declared_functions() == sorted(g.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = g.load_library()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", g.library_path()],
                         capture_output=True, text=True, check=True).stdout
    syms = set(re.findall(r"\bT (gmresir_\w+)", out))
    assert set(_declared_functions()) <= syms


def _c_layout():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "gmresir.h"
int main(void) {
  printf("opts %zu %zu %zu %zu %zu %zu %zu\n", sizeof(gmresir_opts),
         offsetof(gmresir_opts, tau), offsetof(gmresir_opts, imax),
         offsetof(gmresir_opts, berr_target), offsetof(gmresir_opts, scale_pow2),
         offsetof(gmresir_opts, keep_recycle), offsetof(gmresir_opts, ortho));
  printf("timing %zu\n", offsetof(gmresir_opts, timing));
  printf("kstat %zu %zu %zu %zu %zu\n", sizeof(gmresir_kernel_stat),
         offsetof(gmresir_kernel_stat, launches), offsetof(gmresir_kernel_stat, bound),
         offsetof(gmresir_kernel_stat, total_ms), offsetof(gmresir_kernel_stat, work));
  printf("info %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(gmresir_info),
         offsetof(gmresir_info, its), offsetof(gmresir_info, berr),
         offsetof(gmresir_info, singular_col), offsetof(gmresir_info, t_solve_s),
         offsetof(gmresir_info, berr_cw), offsetof(gmresir_info, t_arnoldi_s),
         offsetof(gmresir_info, cycles_persistent), offsetof(gmresir_info, cycles_fallback));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "p.c")
        exe = os.path.join(d, "p")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), c, "-o", exe],
                       check=True)
        return subprocess.run([exe], capture_output=True, text=True, check=True).stdout


def test_struct_layout_matches_header():
    lines = dict(l.split(" ", 1) for l in _c_layout().strip().splitlines())
    o = [int(v) for v in lines["opts"].split()]
    assert o == [ctypes.sizeof(g.Opts), g.Opts.tau.offset, g.Opts.imax.offset,
                 g.Opts.berr_target.offset, g.Opts.scale_pow2.offset,
                 g.Opts.keep_recycle.offset, g.Opts.ortho.offset]
    assert int(lines["timing"]) == g.Opts.timing.offset
    ks = [int(v) for v in lines["kstat"].split()]
    assert ks == [ctypes.sizeof(g.KernelStat), g.KernelStat.launches.offset,
                  g.KernelStat.bound.offset, g.KernelStat.total_ms.offset,
                  g.KernelStat.work.offset]
    i = [int(v) for v in lines["info"].split()]
    assert i == [ctypes.sizeof(g.Info), g.Info.its.offset, g.Info.berr.offset,
                 g.Info.singular_col.offset, g.Info.t_solve_s.offset, g.Info.berr_cw.offset,
                 g.Info.t_arnoldi_s.offset, g.Info.cycles_persistent.offset,
                 g.Info.cycles_fallback.offset]


def test_host_only_entry_points():
    lib = g.load_library()
    o = g.default_opts()
    assert o.struct_size == ctypes.sizeof(g.Opts)
    assert (o.uf, o.u, o.ur, o.m, o.k) == (g.PREC["fp16"], g.PREC["fp32"], g.PREC["fp64"], 30, 10)
    assert o.tau == 1e-4 and o.berr_target == 1e-14 and o.imax == 10
    for st in (0, -1, -2, -3, -4, 1, 2, 3):
        assert lib.gmresir_strerror(st)
    n = ctypes.c_int64(-1)
    abi = ctypes.c_int32(0)
    assert lib.gmresir_query(None, ctypes.byref(n), ctypes.byref(abi)) == -1
    assert abi.value == 3
    lib.gmresir_free(None)          # NULL-safe


def test_invalid_arguments_rejected_before_any_device_call():
    lib = g.load_library()
    out = ctypes.c_void_p()
    o = g.default_opts()
    # NULL matrix
    assert lib.gmresir_factor(None, 10, 10, ctypes.byref(o), None, ctypes.byref(out)) == -1
    assert not out
    # m <= k
    o.m, o.k = 5, 5
    assert lib.gmresir_factor(ctypes.c_void_p(16), 10, 10, ctypes.byref(o), None,
                              ctypes.byref(out)) == -1
    o = g.default_opts()
    o.struct_size = 3
    assert lib.gmresir_factor(ctypes.c_void_p(16), 10, 10, ctypes.byref(o), None,
                              ctypes.byref(out)) == -1
    o = g.default_opts()
    assert lib.gmresir_factor(ctypes.c_void_p(16), 10, 5, ctypes.byref(o), None,
                              ctypes.byref(out)) == -1   # lda < n
    assert b"lda" in lib.gmresir_last_error() or b"invalid" in lib.gmresir_last_error()
