"""Torch-facing calls of the submatrix-method library.

Tensors supply device memory and the current HIP stream; all computation
runs in libsubmat.so. ``invroot`` is differentiable with respect to the
values of A (Daleckii-Krein adjoint in the library).
"""
from __future__ import annotations

import torch

from . import _lib

_PREC = {"f64": _lib.SUBMAT_PREC_F64, "f32_mixed": _lib.SUBMAT_PREC_F32_MIXED,
         "f64_plain": _lib.SUBMAT_PREC_F64_PLAIN}


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


def query_status() -> dict:
    return _lib.submat_query_status(_stream())


def time_phases(rowptr, colind, vals, p=2, precision="f64", grad_x=None) -> dict:
    """Per-phase device time (ms) and launch counts of one forward (and
    adjoint when grad_x is given), direct launches timed with HIP events on
    the current stream."""
    _check_csr(rowptr, colind, vals)
    x = torch.empty_like(vals)
    ga = torch.empty_like(vals) if grad_x is not None else None
    return _lib.submat_time_phases(rowptr.data_ptr(), colind.data_ptr(), vals.data_ptr(), rowptr.numel() - 1,
                                   colind.numel(), int(p), _dtype_code(vals), _prec_code(precision), x.data_ptr(),
                                   grad_x.contiguous().data_ptr() if grad_x is not None else None,
                                   ga.data_ptr() if ga is not None else None, _stream())


class InvRoot(torch.autograd.Function):
    """X.vals = submatrix-method inverse p-th root of A (values on A's
    pattern); gradients flow to A's values only."""

    @staticmethod
    def forward(ctx, rowptr, colind, vals, p, precision, keep_eigvecs):
        saved = None
        if keep_eigvecs:
            nb = saved_bytes(rowptr, colind, vals.dtype, precision)
            saved = torch.empty(max(nb, 8), dtype=torch.uint8, device=vals.device)
        x = invroot_fwd(rowptr, colind, vals, p, precision, saved)
        ctx.save_for_backward(rowptr, colind, vals)
        ctx.p = p
        ctx.precision = precision
        ctx.saved = saved
        return x

    @staticmethod
    def backward(ctx, grad_x):
        rowptr, colind, vals = ctx.saved_tensors
        ga = invroot_bwd(rowptr, colind, vals, grad_x, ctx.p, ctx.precision, ctx.saved)
        ctx.saved = None
        return None, None, ga, None, None, None


def invroot(rowptr, colind, vals, p: int = 2, precision="f64", keep_eigvecs: bool = False) -> torch.Tensor:
    """Differentiable forward: returns X's values on A's pattern."""
    return InvRoot.apply(rowptr, colind, vals, int(p), precision, bool(keep_eigvecs))


def invroot_csr(a: torch.Tensor, p: int = 2, precision="f64") -> torch.Tensor:
    """X for a torch sparse CSR matrix A, sharing A's index tensors (the
    pattern is reused, Section 3.4)."""
    if a.layout != torch.sparse_csr:
        raise ValueError("expected a sparse CSR tensor")
    rowptr = a.crow_indices().to(torch.int32)
    colind = a.col_indices().to(torch.int32)
    x = invroot(rowptr, colind, a.values().contiguous(), p, precision)
    return torch.sparse_csr_tensor(a.crow_indices(), a.col_indices(), x, a.shape)
