"""Randomized-multiplier GENP (Pan & Qian, arXiv:1212.4560) for AMD MI355X.

C = A G with a Gaussian or Gaussian-Toeplitz multiplier, Gaussian elimination
with no pivoting on C, substitutions, X = G Y and FP64 refinement, all in the
HIP library ``libgenp.so`` (C ABI in ``include/genp.h``).

* ``paper_1212_4560_amd.genp``      -- the binding (ctypes) and autograd function
* ``paper_1212_4560_amd.workloads`` -- seeded synthetic inputs
* ``paper_1212_4560_amd.build``     -- hipcc build of the library

Importing the package loads nothing; the binding loads the library on first use.
"""
__version__ = "0.1.0"
