"""FP64 CPU oracle of the NOHAP/OUCS3 compressible-NSE hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product library never does.
It shares no code with the GPU library (see ``nopcs_oracle.c``).

Parity status of each function (what pins it is in ``tests/test_oracle_pins.py``):
  d1 / d1_seg / equiv_row / thomas : pinned (Appendix table, closed forms,
                                     exact rational solves, segment invariance)
  d2                               : pinned (D1 applied twice; transfer function)
  rhs / rhs_points                 : pinned (quiescent state, linear shear,
                                     hydrostatic column, acoustic speed)
  rk4 / rk4_linear                 : pinned (RK4 stability polynomial)
  apply_bc                         : pinned (adiabatic one-sided condition)
"""
from .oracle import *  # noqa: F401,F403
