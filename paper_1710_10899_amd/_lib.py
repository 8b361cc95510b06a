"""ctypes binding of libsubmat.so: the C ABI declared in include/submat.h,
under the same names. Argument marshalling only; every step of the
computation runs in the library's HIP kernels.

Loading fails loudly when the library has not been built: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsubmat.so")

SUBMAT_F64 = 0
SUBMAT_F32 = 1
SUBMAT_PREC_F64 = 0
SUBMAT_PREC_F32_MIXED = 1
SUBMAT_PREC_F64_PLAIN = 2

SUBMAT_OK = 0
SUBMAT_EINVAL = -1
SUBMAT_EPATTERN = -2
SUBMAT_ENODIAG = -3
SUBMAT_ENOMEM = -4
SUBMAT_EHIP = -5
SUBMAT_ETOOBIG = -6
SUBMAT_ESAVED = -7
SUBMAT_EBREAKDOWN = -8
SUBMAT_ENOCONV = -9
SUBMAT_MAX_ORDER = 2048

SUBMAT_FN_INV_ROOT = 0
SUBMAT_FN_ROOT = 1
SUBMAT_FN_POWER = 2

SUBMAT_OPT_KAPPA_MAX = 1
SUBMAT_OPT_USE_GRAPH = 2
SUBMAT_OPT_SMALL_MAX = 3
SUBMAT_OPT_WS_BYTES = 4
SUBMAT_OPT_CLUSTER_TOL = 5
SUBMAT_OPT_TUNE_FILE = 6
SUBMAT_OPT_DETERMINISTIC = 7
SUBMAT_OPT_PLAIN_STRIDE = 8
SUBMAT_OPT_XCD_QUEUES = 9
SUBMAT_NUM_PHASES = 10

PHASES = ["plan-reset", "small-jacobi", "gather", "tridiagonalise", "tridiagonal-eig", "reorthogonalise",
          "back-transform", "apply-column", "adjoint", "fallback"]

# exported symbol -> (restype, argtypes)
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double
SIGNATURES = {
    "submat_matfun_fwd": (ctypes.c_int, [_P, _P, _P, _I32, _I64, _I32, _D, _I32, _I32, _P, _P, _P]),
    "submat_matfun_bwd": (ctypes.c_int, [_P, _P, _P, _I32, _I64, _I32, _D, _I32, _I32, _P, _P, _P, _P]),
    "submat_invroot_fwd": (ctypes.c_int, [_P, _P, _P, _I32, _I64, _I32, _I32, _I32, _P, _P, _P]),
    "submat_invroot_bwd": (ctypes.c_int, [_P, _P, _P, _I32, _I64, _I32, _I32, _I32, _P, _P, _P, _P]),
    "submat_invroot_fwd_noalloc": (ctypes.c_int, [_P, _P, _P, _I32, _I64, _I32, _I32, _I32, _P, _P]),
    "submat_saved_bytes": (_I64, [_P, _P, _I32, _I64, _I32, _I32]),
    "submat_query_status": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "submat_query_counters": (ctypes.c_int, [_P, ctypes.POINTER(_I64), _I32]),
    "submat_set_option": (ctypes.c_int, [_I32, ctypes.c_double]),
    "submat_get_option": (ctypes.c_double, [_I32]),
    "submat_strerror": (ctypes.c_char_p, [_I32]),
    "submat_release": (None, []),
    "submat_release_pattern": (ctypes.c_int, [_P, _P, _I32, _I64]),
    "submat_version": (_I32, []),
    "submat_spmv": (ctypes.c_int, [_P, _P, _P, _I32, _I64, _I32, _P, _P, _P]),
    "submat_residual_norm": (ctypes.c_int, [_P, _P, _P, _P, _I32, _I64, _I32, _I32, _D, ctypes.POINTER(_D),
                                            ctypes.POINTER(_I32), _P]),
    "submat_pcg": (ctypes.c_int, [_P, _P, _P, _P, _I32, _I64, _P, _P, _D, _I32, ctypes.POINTER(_I32),
                                  ctypes.POINTER(_D), ctypes.POINTER(_D), _P]),
    "submat_refine_inverse": (ctypes.c_int, [_P, _P, _P, _P, _I32, _I64, _P, _I32, _D, ctypes.POINTER(_I32),
                                             ctypes.POINTER(_D), _P]),
    "submat_time_phases": (ctypes.c_int, [_P, _P, _P, _I32, _I64, _I32, _D, _I32, _I32, _P, _P, _P, _P,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I32)]),
}

_lib = None


class SubmatError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


def load(path: str | None = None) -> ctypes.CDLL:
    """Loads libsubmat.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built; run `python -m paper_1710_10899_amd.build` "
                           "(there is no CPU fallback)")
    # One HIP runtime per process: torch ships its own libamdhip64 under the
    # soname the library links against, so torch is loaded first and the
    # library binds to that copy (loaded the other way round, torch would
    # run on the system runtime and the tensors it hands over would not be
    # valid in the library's calls).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    if _lib is None:
        return f"status {code}"
    return _lib.submat_strerror(code).decode()


def _check(code: int, where: str) -> None:
    if code != SUBMAT_OK:
        raise SubmatError(code, where)


# ---- same-name wrappers over raw pointers / integers -----------------------

def submat_matfun_fwd(rowptr, colind, vals, n, nnz, fn, param, dtype, precision, x_vals, saved, stream) -> None:
    _check(load().submat_matfun_fwd(rowptr, colind, vals, n, nnz, fn, param, dtype, precision, x_vals, saved,
                                    stream), "submat_matfun_fwd")


def submat_matfun_bwd(rowptr, colind, vals, n, nnz, fn, param, dtype, precision, grad_x, grad_a, saved,
                      stream) -> None:
    _check(load().submat_matfun_bwd(rowptr, colind, vals, n, nnz, fn, param, dtype, precision, grad_x, grad_a,
                                    saved, stream), "submat_matfun_bwd")


def submat_invroot_fwd(rowptr, colind, vals, n, nnz, p, dtype, precision, x_vals, saved, stream) -> None:
    _check(load().submat_invroot_fwd(rowptr, colind, vals, n, nnz, p, dtype, precision, x_vals, saved, stream),
           "submat_invroot_fwd")


def submat_invroot_fwd_noalloc(rowptr, colind, vals, n, nnz, p, dtype, precision, x_vals, stream) -> None:
    _check(load().submat_invroot_fwd_noalloc(rowptr, colind, vals, n, nnz, p, dtype, precision, x_vals, stream),
           "submat_invroot_fwd_noalloc")


def submat_invroot_bwd(rowptr, colind, vals, n, nnz, p, dtype, precision, grad_x, grad_a, saved, stream) -> None:
    _check(load().submat_invroot_bwd(rowptr, colind, vals, n, nnz, p, dtype, precision, grad_x, grad_a, saved,
                                     stream), "submat_invroot_bwd")


def submat_saved_bytes(rowptr, colind, n, nnz, dtype, precision) -> int:
    r = load().submat_saved_bytes(rowptr, colind, n, nnz, dtype, precision)
    if r < 0:
        raise SubmatError(int(r), "submat_saved_bytes")
    return int(r)


def submat_query_status(stream) -> dict:
    a, b, c = _I64(0), _I64(0), _I64(0)
    _check(load().submat_query_status(stream, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "submat_query_status")
    return {"nonpositive": a.value, "fallback": b.value, "unconverged": c.value}


def submat_query_counters(stream, n: int = 4) -> list:
    buf = (_I64 * n)()
    _check(load().submat_query_counters(stream, buf, n), "submat_query_counters")
    return list(buf)


def submat_set_option(key: int, value: float) -> None:
    _check(load().submat_set_option(key, float(value)), "submat_set_option")


def submat_get_option(key: int) -> float:
    return float(load().submat_get_option(key))


def submat_strerror(code: int) -> str:
    return load().submat_strerror(code).decode()


def submat_release() -> None:
    load().submat_release()


def submat_release_pattern(rowptr, colind, n, nnz) -> None:
    _check(load().submat_release_pattern(rowptr, colind, n, nnz), "submat_release_pattern")


def submat_version() -> int:
    return int(load().submat_version())


def submat_spmv(rowptr, colind, vals, n, nnz, trans, x, y, stream) -> None:
    _check(load().submat_spmv(rowptr, colind, vals, n, nnz, trans, x, y, stream), "submat_spmv")


def submat_residual_norm(rowptr, colind, a_vals, x_vals, n, nnz, p, max_iter, tol, stream):
    norm = _D()
    iters = _I32()
    _check(load().submat_residual_norm(rowptr, colind, a_vals, x_vals, n, nnz, p, max_iter, tol,
                                       ctypes.byref(norm), ctypes.byref(iters), stream), "submat_residual_norm")
    return norm.value, iters.value


def submat_pcg(rowptr, colind, a_vals, k_vals, n, nnz, b, x, tol, max_iter, stream) -> dict:
    """Returns {"iters", "relres", "true_relres", "breakdown"}; a breakdown
    is reported in the result, not raised."""
    iters = _I32()
    rel = _D()
    true_rel = _D()
    rc = load().submat_pcg(rowptr, colind, a_vals, k_vals, n, nnz, b, x, tol, max_iter, ctypes.byref(iters),
                           ctypes.byref(rel), ctypes.byref(true_rel), stream)
    if rc not in (SUBMAT_OK, SUBMAT_EBREAKDOWN):
        _check(rc, "submat_pcg")
    return {"iters": iters.value, "relres": rel.value, "true_relres": true_rel.value,
            "breakdown": rc == SUBMAT_EBREAKDOWN}


def submat_refine_inverse(rowptr, colind, a_vals, x_vals, n, nnz, x_dense, max_iter, tol, stream) -> dict:
    """Returns {"iters", "residual", "converged"}; non-convergence is
    reported in the result, not raised."""
    iters = _I32()
    res = _D()
    rc = load().submat_refine_inverse(rowptr, colind, a_vals, x_vals, n, nnz, x_dense, max_iter, tol,
                                      ctypes.byref(iters), ctypes.byref(res), stream)
    if rc not in (SUBMAT_OK, SUBMAT_ENOCONV):
        _check(rc, "submat_refine_inverse")
    return {"iters": iters.value, "residual": res.value, "converged": rc == SUBMAT_OK}


def submat_time_phases(rowptr, colind, vals, n, nnz, fn, param, dtype, precision, x_vals, grad_x, grad_a,
                       stream) -> dict:
    ms = (ctypes.c_double * SUBMAT_NUM_PHASES)()
    nl = (_I32 * SUBMAT_NUM_PHASES)()
    _check(load().submat_time_phases(rowptr, colind, vals, n, nnz, fn, param, dtype, precision, x_vals, grad_x,
                                     grad_a, stream, ms, nl), "submat_time_phases")
    return {PHASES[i]: (ms[i], nl[i]) for i in range(SUBMAT_NUM_PHASES)}
