"""CPU FP64 oracle for the frozen full-metric tangent transport.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package; only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library: it forms A = I - W, C and P explicitly from the paper's definitions and
solves the same systems by other means (Gauss-Seidel directional sweeping to
convergence, dense LU, SuperLU).

Modules
  assembly   face-upwind assembly of W and the calibration c      (Section 3.1, 3.2)
             and the 26-neighbour (cube) stencil variant
  solve      J and J^T by sweeping / dense LU / SuperLU            (Sections 3.6, 4.4)
  diag       graph diagnostics: SCCs, Kahn residual, f_vio, ...    (Sections 3.3-3.5, 4.1-4.2)
  sweep.c    the Gauss-Seidel sweep kernel in plain C              (Section 3.6)

Parity status of each function is stated in its docstring; every function is
pinned by a test under tests/test_oracle_*.py against values or identities the
paper or the mathematics fixes.
"""
from .assembly import assemble, face_coefficients, OracleOperator  # noqa: F401
from .solve import (  # noqa: F401
    build as build_c,
    gs_solve,
    dense_solve,
    superlu_solve,
    apply_J,
    apply_JT,
    apply_JT_summed,
)
from . import diag  # noqa: F401
