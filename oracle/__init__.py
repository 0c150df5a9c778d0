"""CPU oracle for mixed-precision GMRES-IR with Krylov subspace recycling.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library: the only module both sides import is ``synthetic`` (seeded inputs).

What it computes (Oktay & Carson, "Mixed Precision GMRES-based Iterative
Refinement with Recycling"):

* :mod:`oracle.fp` -- rounding to fp16/bf16/fp32 and double-double
  arithmetic (the paper's simulated precisions, Section 3 and Table
  "tab:eps");
* :mod:`oracle.lu` -- GEPP in u_f (the factorisation step of Algorithms 1-3);
* :mod:`oracle.krylov` -- GMRES(m) and GCRO-DR(m, k) (Algorithm "GCRO-DR",
  Section 2);
* :mod:`oracle.refine` -- GMRES-IR (Algorithm 2) and RGMRES-IR (Algorithm 3).

Everything is plain numpy/scipy in float64, with each low-precision result
rounded where the algorithm stores it.

Pins (see ``tests/test_oracle_*.py``) tie each part to facts other than the
oracle itself: unit roundoffs of Table "tab:eps", exhaustive fp16/bf16
round trips, exact rational arithmetic, the prolate condition numbers of
Table "tab:prolate", LAPACK's pivot order, Arnoldi relations, exact GMRES
iteration counts on diagonal operators, exact deflation for recycling, and
backward-error bounds.

Parity unpinned: the paper's iteration-count tables (its MATLAB randsvd
stream, chop configuration, orthogonalisation scheme and stopping rule are
not reproducible), so they serve only as soft context.
"""
from . import fp, krylov, lu, refine  # noqa: F401
from .refine import Options, Info, Factors, factor, solve, gmresir  # noqa: F401
