"""MI355X (gfx950) submatrix-method library: X ~ A^(-1/p) (and the other
spectral functions lambda^(1/p), lambda^alpha) on A's sparsity pattern (Lass
et al., arXiv:1710.10899), with a Daleckii-Krein adjoint and a
mixed-precision form. The computation lives in libsubmat.so (C ABI in
include/submat.h); this package only binds it.
"""
from . import _lib  # noqa: F401
from ._lib import (  # noqa: F401
    SUBMAT_F32,
    SUBMAT_F64,
    SUBMAT_PREC_F32_MIXED,
    SUBMAT_PREC_F64,
    SUBMAT_PREC_F64_PLAIN,
    SubmatError,
)

__all__ = ["invroot", "invroot_fwd", "invroot_bwd", "invroot_csr", "matfun", "matfun_fwd", "matfun_bwd",
           "matfun_csr", "spmv", "residual_norm", "pcg", "refine_inverse", "saved_bytes", "query_status", "time_phases", "MatFun",
           "release_pattern"]


def __getattr__(name):
    # the torch-facing layer is imported on first use so that the ctypes
    # binding can be inspected without importing torch
    if name in __all__:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
