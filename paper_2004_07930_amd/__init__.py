"""MI355X (gfx950) P3 Helmholtz solver with two-level ORAS-preconditioned block FGMRES.

The compute path is libhz.so (hand-written HIP kernels behind the C ABI in include/hz.h);
this package only loads it and marshals arguments (see hz.py).
"""
from .hz import (HZ_BC_DIRICHLET, HZ_BC_IMPEDANCE, HZ_MEM_DEVICE, HZ_MEM_HOST, HZ_PREC_C128,  # noqa: F401
                 HZ_PREC_MIXED, Context, HzError, load)
