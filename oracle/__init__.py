"""FP64 CPU oracle for explicit f-x poststack depth migration (TEST INFRASTRUCTURE).

This package exists only to check the GPU path.  The test suite, the smoke
check and the CPU-baseline leg of ``bench.py`` are its only callers; the product
library never imports, links or runs it, and it imports nothing from the
product package.  The arithmetic lives in ``oracle.c`` (plain C, IEEE double,
``-ffp-contract=off``, OpenMP over frequencies); this module only builds and
marshals it.

Functions follow the paper (Shawahna, Salam & Al-Mouhamed, arXiv 1912.05529):

* :func:`design_table` -- predesigned FIR extrapolator bank (Sec. II, Sec. III).
  The paper gives no design method; this is a weighted least-squares fit to the
  phase shift with reweighting and a rigorous stability scale.
* :func:`table_index` -- the table look-up of Algorithm 1 (nearest entry in
  omega/v).
* :func:`extrapolate` -- Eq. (1), literally, depth step after depth step.
* :func:`image` -- depth row = Re of the sum over frequencies (Algorithm 1).
* :func:`migrate` -- Algorithm 1 end to end on an f-x section.
* :func:`demigrate` -- exact adjoint of :func:`migrate`.
* :func:`design_table_2d`, :func:`migrate3d` -- the 3-D extension (Sec. II):
  circularly symmetric 2-D extrapolators and the 2-D form of Eq. (1).
* :func:`transform_t` -- the transform along t that precedes the depth loop
  (Algorithm 1, first step), evaluated directly at the requested frequencies.

Parity status: every function above is pinned by a CPU test against a closed
form, a textbook routine, an invariant or brute force (``tests/test_oracle_*``).
"""
from .core import (  # noqa: F401
    OrcDesc,
    build,
    demigrate,
    design_table,
    design_table_2d,
    extrapolate,
    image,
    load,
    migrate,
    migrate3d,
    num_threads,
    table_index,
    transform_t,
)
