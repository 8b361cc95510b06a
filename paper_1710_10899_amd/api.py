"""Torch-facing calls of the submatrix-method library.

Tensors supply device memory and the current HIP stream; all computation
runs in libsubmat.so. ``matfun`` (any of the library's spectral functions)
and ``invroot`` (the inverse p-th root) are differentiable with respect to
the values of A (Daleckii-Krein adjoint in the library).

Spectral functions, by name -> library code (the parameter is p for the two
roots, the exponent alpha for a real power):
  "inv_root"  lambda^(-1/p)   the paper's main case (Sections 3-4)
  "root"      lambda^(1/p)    positive p-th roots (Section 4, other matrix operations)
  "power"     lambda^alpha    any real power
"""
from __future__ import annotations

import weakref

import torch

from . import _lib

_PREC = {"f64": _lib.SUBMAT_PREC_F64, "f32_mixed": _lib.SUBMAT_PREC_F32_MIXED,
         "f64_plain": _lib.SUBMAT_PREC_F64_PLAIN}


_FN = {"inv_root": _lib.SUBMAT_FN_INV_ROOT, "root": _lib.SUBMAT_FN_ROOT, "power": _lib.SUBMAT_FN_POWER}


def _fn_code(fn) -> int:
    if isinstance(fn, int):
        return fn
    try:
        return _FN[fn]
    except KeyError:
        raise ValueError(f"fn must be one of {sorted(_FN)}") from None


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return _lib.SUBMAT_F64
    if t.dtype == torch.float32:
        return _lib.SUBMAT_F32
    raise TypeError(f"values must be float64 or float32, got {t.dtype}")


def _prec_code(precision) -> int:
    if isinstance(precision, int):
        return precision
    try:
        return _PREC[precision]
    except KeyError:
        raise ValueError(f"precision must be one of {sorted(_PREC)}") from None


def _check_csr(rowptr: torch.Tensor, colind: torch.Tensor, vals: torch.Tensor) -> None:
    for name, t in (("rowptr", rowptr), ("colind", colind), ("vals", vals)):
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor (the library has no CPU path)")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    if rowptr.dtype != torch.int32 or colind.dtype != torch.int32:
        raise TypeError("rowptr and colind must be int32")
    if vals.numel() != colind.numel():
        raise ValueError("vals and colind must have nnz entries")


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def saved_bytes(rowptr, colind, dtype=torch.float64, precision="f64") -> int:
    n = rowptr.numel() - 1
    code = _lib.SUBMAT_F64 if dtype == torch.float64 else _lib.SUBMAT_F32
    return _lib.submat_saved_bytes(rowptr.data_ptr(), colind.data_ptr(), n, colind.numel(), code,
                                   _prec_code(precision))


def matfun_fwd(rowptr, colind, vals, fn="inv_root", param: float = 2, precision="f64",
               saved: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """X.vals with X = f(A) by the submatrix method, on A's pattern."""
    _check_csr(rowptr, colind, vals)
    x = torch.empty_like(vals) if out is None else out
    _lib.submat_matfun_fwd(rowptr.data_ptr(), colind.data_ptr(), vals.data_ptr(), rowptr.numel() - 1,
                           colind.numel(), _fn_code(fn), float(param), _dtype_code(vals), _prec_code(precision),
                           x.data_ptr(), saved.data_ptr() if saved is not None else None, _stream())
    return x


def matfun_bwd(rowptr, colind, vals, grad_x, fn="inv_root", param: float = 2, precision="f64",
               saved: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """dL/dA.vals for L = sum(grad_x * X.vals)."""
    _check_csr(rowptr, colind, vals)
    grad_x = grad_x.contiguous()
    if grad_x.dtype != vals.dtype or grad_x.numel() != vals.numel():
        raise ValueError("grad_x must match vals in dtype and size")
    ga = torch.empty_like(vals) if out is None else out
    _lib.submat_matfun_bwd(rowptr.data_ptr(), colind.data_ptr(), vals.data_ptr(), rowptr.numel() - 1,
                           colind.numel(), _fn_code(fn), float(param), _dtype_code(vals), _prec_code(precision),
                           grad_x.data_ptr(), ga.data_ptr(), saved.data_ptr() if saved is not None else None,
                           _stream())
    return ga


def invroot_fwd(rowptr, colind, vals, p: int = 2, precision="f64", saved: torch.Tensor | None = None,
                out: torch.Tensor | None = None) -> torch.Tensor:
    _check_csr(rowptr, colind, vals)
    x = torch.empty_like(vals) if out is None else out
    _lib.submat_invroot_fwd(rowptr.data_ptr(), colind.data_ptr(), vals.data_ptr(), rowptr.numel() - 1,
                            colind.numel(), int(p), _dtype_code(vals), _prec_code(precision), x.data_ptr(),
                            saved.data_ptr() if saved is not None else None, _stream())
    return x


def invroot_bwd(rowptr, colind, vals, grad_x, p: int = 2, precision="f64", saved: torch.Tensor | None = None,
                out: torch.Tensor | None = None) -> torch.Tensor:
    _check_csr(rowptr, colind, vals)
    grad_x = grad_x.contiguous()
    if grad_x.dtype != vals.dtype or grad_x.numel() != vals.numel():
        raise ValueError("grad_x must match vals in dtype and size")
    ga = torch.empty_like(vals) if out is None else out
    _lib.submat_invroot_bwd(rowptr.data_ptr(), colind.data_ptr(), vals.data_ptr(), rowptr.numel() - 1,
                            colind.numel(), int(p), _dtype_code(vals), _prec_code(precision), grad_x.data_ptr(),
                            ga.data_ptr(), saved.data_ptr() if saved is not None else None, _stream())
    return ga


def _check_f64_vec(name, v, n):
    if not v.is_cuda or v.dtype != torch.float64 or not v.is_contiguous() or v.numel() != n:
        raise ValueError(f"{name} must be a contiguous float64 device vector of {n} entries")


def spmv(rowptr, colind, vals, x, trans: bool = False, out: torch.Tensor | None = None) -> torch.Tensor:
    """y = M x (trans=False) or M^T x for the CSR matrix M with row i holding
    vals[rowptr[i]:rowptr[i+1]] at columns colind[...]. For the column-based
    result X of matfun_fwd, X^T x is trans=False and X x is trans=True."""
    _check_csr(rowptr, colind, vals)
    n = rowptr.numel() - 1
    if vals.dtype != torch.float64:
        raise TypeError("spmv takes float64 values")
    _check_f64_vec("x", x, n)
    y = torch.empty_like(x) if out is None else out
    _lib.submat_spmv(rowptr.data_ptr(), colind.data_ptr(), vals.data_ptr(), n, colind.numel(), int(bool(trans)),
                     x.data_ptr(), y.data_ptr(), _stream())
    return y


def residual_norm(rowptr, colind, a_vals, x_vals, p: int = 2, max_iter: int = 300, tol: float = 1e-10):
    """||X^p A - I||_2 (Section 4.1) by Lanczos on R^T R in the library;
    returns (norm, lanczos_steps)."""
    _check_csr(rowptr, colind, a_vals)
    _check_csr(rowptr, colind, x_vals)
    if a_vals.dtype != torch.float64 or x_vals.dtype != torch.float64:
        raise TypeError("residual_norm takes float64 values")
    return _lib.submat_residual_norm(rowptr.data_ptr(), colind.data_ptr(), a_vals.data_ptr(), x_vals.data_ptr(),
                                     rowptr.numel() - 1, colind.numel(), int(p), int(max_iter), float(tol),
                                     _stream())


def pcg(rowptr, colind, a_vals, b, k_vals=None, tol: float = 1e-6, max_iter: int | None = None,
        out: torch.Tensor | None = None):
    """Solve A x = b by CG on K^T A K y = K^T b, x = K y (Section 4.4), with
    K the column-based values of an approximate A^(-1/2) (None: plain CG).
    max_iter defaults to 2 n. Returns (x, info) with info = {"iters",
    "relres", "true_relres", "breakdown"}."""
    _check_csr(rowptr, colind, a_vals)
    n = rowptr.numel() - 1
    if a_vals.dtype != torch.float64:
        raise TypeError("pcg takes float64 values")
    _check_f64_vec("b", b, n)
    if k_vals is not None:
        _check_csr(rowptr, colind, k_vals)
        if k_vals.dtype != torch.float64:
            raise TypeError("pcg takes float64 values")
    x = torch.empty_like(b) if out is None else out
    info = _lib.submat_pcg(rowptr.data_ptr(), colind.data_ptr(), a_vals.data_ptr(),
                           k_vals.data_ptr() if k_vals is not None else None, n, colind.numel(), b.data_ptr(),
                           x.data_ptr(), float(tol), int(2 * n if max_iter is None else max_iter), _stream())
    return x, info


def refine_inverse(rowptr, colind, a_vals, x_vals, max_iter: int = 20, tol: float = 1e-14,
                   out: torch.Tensor | None = None):
    """Newton-Schulz refinement of the submatrix-method inverse (p = 1)
    seeded with x_vals (Section 4.5); returns (dense row-major X, info)."""
    _check_csr(rowptr, colind, a_vals)
    _check_csr(rowptr, colind, x_vals)
    if a_vals.dtype != torch.float64 or x_vals.dtype != torch.float64:
        raise TypeError("refine_inverse takes float64 values")
    n = rowptr.numel() - 1
    xd = torch.empty((n, n), dtype=torch.float64, device=a_vals.device) if out is None else out
    if xd.shape != (n, n) or not xd.is_contiguous() or xd.dtype != torch.float64:
        raise ValueError("out must be a contiguous float64 n x n tensor")
    info = _lib.submat_refine_inverse(rowptr.data_ptr(), colind.data_ptr(), a_vals.data_ptr(), x_vals.data_ptr(), n,
                                      colind.numel(), xd.data_ptr(), int(max_iter), float(tol), _stream())
    return xd, info


def query_status() -> dict:
    return _lib.submat_query_status(_stream())


def time_phases(rowptr, colind, vals, p=2, precision="f64", grad_x=None, fn="inv_root") -> dict:
    """Per-phase device time (ms) and launch counts of one forward (and
    adjoint when grad_x is given), direct launches timed with HIP events on
    the current stream; `p` is the function's parameter."""
    _check_csr(rowptr, colind, vals)
    x = torch.empty_like(vals)
    ga = torch.empty_like(vals) if grad_x is not None else None
    return _lib.submat_time_phases(rowptr.data_ptr(), colind.data_ptr(), vals.data_ptr(), rowptr.numel() - 1,
                                   colind.numel(), _fn_code(fn), float(p), _dtype_code(vals), _prec_code(precision),
                                   x.data_ptr(), grad_x.contiguous().data_ptr() if grad_x is not None else None,
                                   ga.data_ptr() if ga is not None else None, _stream())


class MatFun(torch.autograd.Function):
    """X.vals = submatrix-method f(A) (values on A's pattern); gradients
    flow to A's values only."""

    @staticmethod
    def forward(ctx, rowptr, colind, vals, fn, param, precision, keep_eigvecs):
        saved = None
        if keep_eigvecs:
            nb = saved_bytes(rowptr, colind, vals.dtype, precision)
            saved = torch.empty(max(nb, 8), dtype=torch.uint8, device=vals.device)
        x = matfun_fwd(rowptr, colind, vals, fn, param, precision, saved)
        ctx.save_for_backward(rowptr, colind, vals)
        ctx.fn = fn
        ctx.param = param
        ctx.precision = precision
        ctx.saved = saved
        return x

    @staticmethod
    def backward(ctx, grad_x):
        rowptr, colind, vals = ctx.saved_tensors
        ga = matfun_bwd(rowptr, colind, vals, grad_x, ctx.fn, ctx.param, ctx.precision, ctx.saved)
        ctx.saved = None
        return None, None, ga, None, None, None, None


def matfun(rowptr, colind, vals, fn="inv_root", param: float = 2, precision="f64",
           keep_eigvecs: bool = False) -> torch.Tensor:
    """Differentiable forward of f(A): returns X's values on A's pattern."""
    return MatFun.apply(rowptr, colind, vals, _fn_code(fn), float(param), precision, bool(keep_eigvecs))


def invroot(rowptr, colind, vals, p: int = 2, precision="f64", keep_eigvecs: bool = False) -> torch.Tensor:
    """Differentiable forward of A^(-1/p): returns X's values on A's pattern."""
    return MatFun.apply(rowptr, colind, vals, _lib.SUBMAT_FN_INV_ROOT, float(int(p)), precision,
                        bool(keep_eigvecs))


def release_pattern(rowptr: torch.Tensor, colind: torch.Tensor) -> None:
    """Drops the library's cached plan for this pattern (call it before the
    index tensors are freed or changed when another pattern of the same n
    and nnz may take their addresses)."""
    _lib.submat_release_pattern(rowptr.data_ptr(), colind.data_ptr(), rowptr.numel() - 1, colind.numel())


# int32 index tensors of the sparse CSR tensors passed to matfun_csr, by id()
# of the sparse tensor: (weak reference to it, rowptr, colind). A finalizer
# drops the entry and the library's plan for those addresses when the sparse
# tensor goes away, so that a later pattern that reuses the addresses never
# meets a stale plan.
_CSR_INDEX = {}


def _forget_csr(key, rp_ptr, ci_ptr, n, nnz):
    _CSR_INDEX.pop(key, None)
    if _lib._lib is not None:
        _lib.submat_release_pattern(rp_ptr, ci_ptr, n, nnz)


def _csr_index32(a: torch.Tensor):
    """(rowptr, colind) of a sparse CSR tensor as int32 device tensors whose
    addresses stay fixed while `a` lives, and whose plan is released when it
    dies."""
    key = id(a)
    hit = _CSR_INDEX.get(key)
    if hit is not None and hit[0]() is a:
        return hit[1], hit[2]
    crow, col = a.crow_indices(), a.col_indices()
    rowptr = crow if crow.dtype == torch.int32 and crow.is_contiguous() else crow.to(torch.int32).contiguous()
    colind = col if col.dtype == torch.int32 and col.is_contiguous() else col.to(torch.int32).contiguous()
    _CSR_INDEX[key] = (weakref.ref(a), rowptr, colind)
    weakref.finalize(a, _forget_csr, key, rowptr.data_ptr(), colind.data_ptr(), rowptr.numel() - 1,
                     colind.numel())
    return rowptr, colind


def invroot_csr(a: torch.Tensor, p: int = 2, precision="f64") -> torch.Tensor:
    """X for a torch sparse CSR matrix A, sharing A's index tensors (the
    pattern is reused, Section 3.4)."""
    return matfun_csr(a, "inv_root", p, precision)


def matfun_csr(a: torch.Tensor, fn="inv_root", param: float = 2, precision="f64") -> torch.Tensor:
    """f(A) for a torch sparse CSR matrix A, on A's pattern and index tensors."""
    if a.layout != torch.sparse_csr:
        raise ValueError("expected a sparse CSR tensor")
    rowptr, colind = _csr_index32(a)
    x = matfun(rowptr, colind, a.values().contiguous(), fn, param, precision)
    return torch.sparse_csr_tensor(a.crow_indices(), a.col_indices(), x, a.shape)
