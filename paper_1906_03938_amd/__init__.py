"""MI355X-native node sweep of the contour / Chebyshev rational approximation method for
boundary-element acoustic eigenproblems T(kappa) x = 0 (arXiv 1906.03938).

The numerical work runs in libbemrat.so (HIP kernels for gfx950, C ABI in
include/bemrat.h); this package is its ctypes binding plus the host driver that
orchestrates sweeps into eigenvalues.
"""
from ._lib import (  # noqa: F401
    FORM_AUTO,
    FORM_CHEB,
    FORM_DIRECT,
    FORM_EXPAND,
    NF_AUTO,
    NF_NODES,
    PREC_BF16,
    PREC_F16,
    PREC_F32,
    PREC_F64,
    Batch,
    BemError,
    Mesh,
    cheb_nodes,
    contour_nodes,
    lib,
    stream_status,
)
