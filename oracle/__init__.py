"""CPU FP64 oracle for the interior point method of Pearson, Porcelli and Stoll
(arXiv 1806.05896) applied to the finite-difference form of the sparse,
box-constrained optimal control problem.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU path is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product library never does,
and it shares no code with it.

Contents
  fd.py   discrete operators (Sec. 2, eq. (pb_fe)) as SciPy sparse matrices,
          boundary data folded into the right-hand side.
  ipm.py  the interior point path-following loop (Appendix, Algorithm A.1)
          with a sparse direct solve of the reduced Newton system (Sec. 3,
          eq. (NewtonSystem)), multiplier recovery (eqs. (zupdate1)-(zupdate4)),
          feasibility and complementarity measures (eqs. (prdu), (gap)).

Every function cites the passage it follows.  Readings taken where the paper
is silent or garbled are listed in the module docstrings.
"""
from .fd import operator_matrix, rhs_offset, Discretization, discretize  # noqa: F401
from .ipm import IPMOptions, IPMResult, IPMState, solve, newton_matrix, newton_rhs, newton_solve  # noqa: F401
