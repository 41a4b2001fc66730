"""CPU oracle for the GCG eigensolver hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product path (``paper_2111_06552_amd``) never imports it, and it
imports nothing from the product path: the two share no code.  The only
common import is ``workloads`` (seeded input generation, no method arithmetic).

Everything here is plain, slow and FP64: numpy arrays, matrix products as the
only library primitive, and a small C file (``csrc/jacobi.c``, cyclic Jacobi)
for dense symmetric eigendecompositions.  There is no LAPACK call anywhere in
this package.  Each function states the passage of the paper (arXiv
2111.06552, "GCGE: A package for solving large scale eigenvalue problems by
parallel block damping inverse power method") that it follows.

Parity status of each function is listed in :data:`PINS`; every function is
pinned by at least one check that does not reuse its own formula (closed
forms, brute force, invariants) in ``tests/test_oracle_pins.py`` and
``tests/test_oracle_amg_pins.py``.
"""
from .core import *  # noqa: F401,F403
from .core import PINS  # noqa: F401
from . import amg  # noqa: F401
