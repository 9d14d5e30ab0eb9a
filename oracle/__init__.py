"""CPU FP64 oracle for the P3 Helmholtz / two-level ORAS-FGMRES solver.

TEST INFRASTRUCTURE ONLY.  Only tests/, the graft smoke check and bench.py's CPU
baseline leg import this package; the solver library and its Python binding never do,
and share no code with it.  It is a plain, slow, obviously correct NumPy / SciPy
implementation that follows the paper's equations step by step:

  p3      reference P3 element, exact rational integrals
  fem     dof numbering, element matrices, global assembly, Dirichlet rows
  rhs     point-source and plane-wave loads
  ddm     overlap, partition of unity, local Robin operators (SuperLU), coarse Z, E (LU)
  krylov  block FGMRES(m) with CGS2, dense direct solve

Parity status: every function is pinned by tests/test_oracle_*.py against closed forms,
invariants, exact identities or library routines (see each test's docstring).
"""
from . import ddm, fem, krylov, p3, rhs  # noqa: F401
