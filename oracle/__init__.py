"""Oracle: a plain, slow, FP64 CPU reference for the node sweep and the eigen-extraction
of the contour / Chebyshev rational approximation method (arXiv 1906.03938).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import, call, link or execute anything in this directory.  It shares no code
with the HIP implementation and never imports the product package.

  bem_oracle.c  -- the BEM operator T(kappa): geometry, Radon's 7-point rule, Green's
                   function, exact polar self term, dense and matrix-free application.
  _clib.py      -- ctypes wrappers and the gcc build of bem_oracle.c.
  method.py     -- nodes and weights, sweep outputs, linearisations, Algorithms 1 and 3,
                   brute-force references (MSLP, argument principle).
"""
from . import _clib
from ._clib import build  # noqa: F401
from . import method  # noqa: F401
