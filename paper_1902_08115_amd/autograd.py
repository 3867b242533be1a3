"""Differentiable dgemm and lower Cholesky on batched column-major FP64 GPU
tensors (torch.autograd.Function wrappers of the C ABI).

Forward and backward run entirely in the library's HIP kernels; torch only
allocates the outputs and supplies the stream.  Tensors follow blas.py's
layout: (batch, rows, cols) with stride(-2) == 1.

  dgemm(A, B, transa, transb, alpha)  C = alpha * op(A) op(B)
        backward: the forward kernels with swapped transposition flags
        (mb_dgemm_backward_strided_batched)
  cholesky(A)                         L = chol(A), lower, upper triangle zero
        backward: the Cholesky adjoint (mb_dpotrf_l_backward_strided_batched),
        symmetric gradient convention
  cholesky_product(A, B)              C = chol(A) B (the composition)
"""
from __future__ import annotations

import torch

from . import _lib, blas
from .blas import _layout, _raise, _stream


def colmajor(X: torch.Tensor) -> torch.Tensor:
    """X itself when already column-major per instance, else a column-major copy."""
    if X.dim() == 3 and (X.shape[-2] <= 1 or X.stride(-2) == 1) and X.stride(-1) >= max(
            1, X.shape[-2]) and (X.shape[0] <= 1 or X.stride(0) >= X.shape[-2] * X.shape[-1]):
        return X
    out = blas.colmajor_empty(X.shape[0], X.shape[1], X.shape[2], device=X.device)
    out.copy_(X)
    return out


def _check(name: str, X: torch.Tensor):
    if X.dtype != torch.float64 or not X.is_cuda or X.dim() != 3:
        raise ValueError(f"{name} must be a 3-D float64 CUDA tensor (batch, rows, cols)")


class Dgemm(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, transa: str, transb: str, alpha: float):
        _check("A", A)
        _check("B", B)
        A, B = colmajor(A), colmajor(B)
        batch = A.shape[0]
        m = A.shape[1] if transa in "Nn" else A.shape[2]
        k = A.shape[2] if transa in "Nn" else A.shape[1]
        n = B.shape[2] if transb in "Nn" else B.shape[1]
        C = blas.colmajor_empty(batch, m, n, device=A.device)
        blas.dgemm_strided_batched(transa, transb, alpha, A, B, 0.0, C)
        ctx.save_for_backward(A, B)
        ctx.args = (transa, transb, alpha, m, n, k)
        return C

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        transa, transb, alpha, m, n, k = ctx.args
        dC = colmajor(dC)
        batch = A.shape[0]
        dA = blas.colmajor_empty(batch, A.shape[1], A.shape[2], device=A.device) \
            if ctx.needs_input_grad[0] else None
        dB = blas.colmajor_empty(batch, B.shape[1], B.shape[2], device=B.device) \
            if ctx.needs_input_grad[1] else None
        lda, sA = _layout(A, "A", True)
        ldb, sB = _layout(B, "B", True)
        lddc, sdC = _layout(dC, "dC", True)
        ldda, sdA = _layout(dA, "dA", True) if dA is not None else (max(1, A.shape[1]), 0)
        lddb, sdB = _layout(dB, "dB", True) if dB is not None else (max(1, B.shape[1]), 0)
        st = _lib.dgemm_backward_strided_batched(
            transa, transb, m, n, k, alpha, A.data_ptr(), lda, sA, B.data_ptr(), ldb, sB,
            dC.data_ptr(), lddc, sdC, dA.data_ptr() if dA is not None else None, ldda, sdA,
            dB.data_ptr() if dB is not None else None, lddb, sdB, batch, _stream(None))
        _raise("mb_dgemm_backward_strided_batched", st)
        return dA, dB, None, None, None


class Cholesky(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A):
        _check("A", A)
        batch, n, n2 = A.shape
        if n != n2:
            raise ValueError("A must be square")
        L = blas.colmajor_empty(batch, n, n, device=A.device)
        L.copy_(A)
        info = blas.dpotrf_strided_batched(L)
        ld, sL = _layout(L, "L", True)
        if n > 1:
            # zero the strict upper triangle (dlaset on the (n-1) x (n-1)
            # block that starts at column 1)
            st = _lib.dlaset_strided_batched("U", n - 1, n - 1, 0.0, 0.0,
                                             L.data_ptr() + 8 * ld, ld, sL, batch, _stream(None))
            _raise("mb_dlaset_strided_batched", st)
        bad = torch.nonzero(info).flatten()
        if bad.numel():
            b = int(bad[0])
            raise torch.linalg.LinAlgError(
                f"instance {b}: leading minor of order {int(info[b])} is not positive definite")
        ctx.save_for_backward(L)
        return L

    @staticmethod
    def backward(ctx, Lbar):
        (L,) = ctx.saved_tensors
        Lbar = colmajor(Lbar)
        batch, n, _ = L.shape
        Abar = blas.colmajor_empty(batch, n, n, device=L.device)
        ldl, sL = _layout(L, "L", True)
        ldlb, sLb = _layout(Lbar, "Lbar", True)
        ldab, sAb = _layout(Abar, "Abar", True)
        st = _lib.dpotrf_l_backward_strided_batched(n, L.data_ptr(), ldl, sL, Lbar.data_ptr(),
                                                    ldlb, sLb, Abar.data_ptr(), ldab, sAb, batch,
                                                    _stream(None))
        _raise("mb_dpotrf_l_backward_strided_batched", st)
        return Abar


def dgemm(A, B, transa: str = "N", transb: str = "N", alpha: float = 1.0):
    return Dgemm.apply(A, B, transa, transb, float(alpha))


def cholesky(A):
    return Cholesky.apply(A)


def cholesky_product(A, B):
    """C = chol(A) B, differentiable in A (symmetric gradient) and B."""
    return dgemm(cholesky(A), B)
