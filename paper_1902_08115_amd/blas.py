"""Torch-facing wrappers of the mi355blas C ABI (memory and streams only).

Tensors must already be column-major FP64 on the GPU: a matrix is a 2-D
tensor with stride(-2) == 1 and stride(-1) == ld >= rows; a strided batch is
a 3-D tensor (batch, rows, cols) with the same per-instance layout and
stride(0) as the instance stride.  Nothing is copied or converted behind the
caller's back: a tensor in any other layout raises.  ``colmajor_empty`` and
``colmajor_from_numpy`` build conforming tensors.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import MbError, VARIANT_AUTO, VARIANT_DIRECT, VARIANT_PACKED, VARIANT_REGTILE  # noqa: F401


def _stream(stream) -> int:
    return (stream if stream is not None else torch.cuda.current_stream()).cuda_stream


def _layout(X: torch.Tensor, name: str, batched: bool):
    """Return (ld, instance_stride) of a column-major FP64 CUDA tensor."""
    if X.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not X.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if X.dim() != (3 if batched else 2):
        raise ValueError(f"{name} must be {'3' if batched else '2'}-D")
    rows, cols = X.shape[-2], X.shape[-1]
    s_r, s_c = X.stride(-2), X.stride(-1)
    if rows > 1 and s_r != 1:
        raise ValueError(f"{name} is not column-major (stride(-2) must be 1)")
    ld = s_c if cols > 1 else max(1, rows, s_c)
    if ld < max(1, rows):
        raise ValueError(f"{name}: leading dimension {ld} < rows {rows}")
    return ld, (X.stride(0) if batched else 0)


def _raise(fn, st):
    if st != _lib.MB_OK:
        raise MbError(fn, st)


def colmajor_empty(batch, rows, cols, ld=None, device="cuda", fill=None):
    """Uninitialised (or ``fill``-ed) column-major batch tensor (batch, rows, cols)."""
    ld = max(1, rows) if ld is None else ld
    base = torch.empty((batch, max(cols, 1), ld), dtype=torch.float64, device=device)
    if fill is not None:
        base.fill_(fill)
    return base.transpose(1, 2)[:, :rows, :cols]


def colmajor_from_numpy(X, rows, device="cuda"):
    """Device copy of a numpy batch in the (batch, cols, ld) column-major
    buffer layout; returns the (batch, rows, cols) view."""
    t = torch.from_numpy(X).to(device)
    return t.transpose(1, 2)[:, :rows, :]


def dgemm(transa, transb, alpha, A, B, beta, C, stream=None):
    """C <= alpha*op(A)*op(B) + beta*C for 2-D column-major tensors."""
    lda, _ = _layout(A, "A", False)
    ldb, _ = _layout(B, "B", False)
    ldc, _ = _layout(C, "C", False)
    m, n = C.shape
    k = A.shape[1] if transa in "Nn" else A.shape[0]
    st = _lib.dgemm(transa, transb, m, n, k, alpha, A.data_ptr(), lda, B.data_ptr(), ldb, beta,
                    C.data_ptr(), ldc, _stream(stream))
    _raise("mb_dgemm", st)
    return C


def dgemm_strided_batched(transa, transb, alpha, A, B, beta, C, variant=None, stream=None):
    """Strided batch over the leading dimension of 3-D column-major tensors."""
    lda, sA = _layout(A, "A", True)
    ldb, sB = _layout(B, "B", True)
    ldc, sC = _layout(C, "C", True)
    batch, m, n = C.shape
    k = A.shape[2] if transa in "Nn" else A.shape[1]
    st = _lib.dgemm_strided_batched(transa, transb, m, n, k, alpha, A.data_ptr(), lda, sA,
                                    B.data_ptr(), ldb, sB, beta, C.data_ptr(), ldc, sC, batch,
                                    _stream(stream), variant)
    _raise("mb_dgemm_strided_batched", st)
    return C


def pointer_array(X: torch.Tensor) -> torch.Tensor:
    """Device array of the instance base pointers of a batch tensor."""
    base = X.data_ptr()
    idx = torch.arange(X.shape[0], dtype=torch.int64)
    return (base + idx * X.stride(0) * 8).to(X.device)


def dgemm_batched(transa, transb, m, n, k, alpha, Aptr, lda, Bptr, ldb, beta, Cptr, ldc, batch,
                  variant=None, stream=None):
    """Pointer-array batch; Aptr/Bptr/Cptr are int64 device tensors of addresses."""
    st = _lib.dgemm_batched(transa, transb, m, n, k, alpha, Aptr.data_ptr(), lda, Bptr.data_ptr(),
                            ldb, beta, Cptr.data_ptr(), ldc, batch, _stream(stream), variant)
    _raise("mb_dgemm_batched", st)


def _check_info(info, stream):
    """check=True: wait for the stream and raise on any non-zero info (the
    behaviour of torch.linalg.cholesky_ex(check_errors=True))."""
    (stream if stream is not None else torch.cuda.current_stream()).synchronize()
    bad = torch.nonzero(info != 0)
    if bad.numel():
        b = int(bad[0, 0]) if bad.dim() > 1 else int(bad[0])
        j = int(info.reshape(-1)[b])
        raise torch.linalg.LinAlgError(
            f"dpotrf: instance {b}: the leading minor of order {j} is not positive definite")


def dpotrf(A, info=None, stream=None, check=False):
    """Lower Cholesky in place on a 2-D column-major tensor; returns the
    device info tensor (shape (1,), int32) -- valid after the stream completes.
    check=True synchronizes and raises torch.linalg.LinAlgError when info != 0."""
    lda, _ = _layout(A, "A", False)
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=A.device)
    st = _lib.dpotrf("L", n, A.data_ptr(), lda, info.data_ptr(), _stream(stream))
    _raise("mb_dpotrf", st)
    if check:
        _check_info(info, stream)
    return info


def dpotrf_strided_batched(A, info=None, stream=None, check=False):
    """Batched form of dpotrf over a 3-D column-major tensor (see dpotrf)."""
    lda, sA = _layout(A, "A", True)
    batch, n, n2 = A.shape
    if n != n2:
        raise ValueError("A must be square")
    if info is None:
        info = torch.empty(max(batch, 1), dtype=torch.int32, device=A.device)[:batch]
    st = _lib.dpotrf_strided_batched("L", n, A.data_ptr(), lda, sA, info.data_ptr(), batch,
                                     _stream(stream))
    _raise("mb_dpotrf_strided_batched", st)
    if check:
        _check_info(info, stream)
    return info


def dpotrf_batched(Aptr, n, lda, batch, info=None, stream=None):
    if info is None:
        info = torch.empty(max(batch, 1), dtype=torch.int32, device=Aptr.device)[:batch]
    st = _lib.dpotrf_batched("L", n, Aptr.data_ptr(), lda, info.data_ptr(), batch,
                             _stream(stream))
    _raise("mb_dpotrf_batched", st)
    return info


def _stages(X: torch.Tensor, name: str, rows: int, cols: int):
    """(ld, stage stride, problem stride) of a (batch, N, rows, cols) tensor of
    column-major FP64 matrices."""
    if X.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not X.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if X.dim() != 4 or tuple(X.shape[2:]) != (rows, cols):
        raise ValueError(f"{name} must be (batch, N, {rows}, {cols})")
    if rows > 1 and X.stride(2) != 1:
        raise ValueError(f"{name} is not column-major (stride(2) must be 1)")
    ld = X.stride(3) if cols > 1 else max(1, rows, X.stride(3))
    return ld, X.stride(1), X.stride(0)


def riccati_workspace(nx, nu, batch, device="cuda"):
    """A workspace tensor sized by mb_riccati_workspace_size (full occupancy)."""
    st, nbytes = _lib.riccati_workspace_size(nx, nu, batch)
    _raise("mb_riccati_workspace_size", st)
    return torch.empty(max(1, (nbytes + 7) // 8), dtype=torch.float64, device=device)


def riccati(BAt, RSQ, QN, nu, F=None, LN=None, info=None, work=None, stream=None):
    """Batched factorized Riccati recursion (Sec. 5.2).

    BAt (batch, N, m, nx), RSQ (batch, N, m, m), QN (batch, nx, nx): column-
    major FP64 GPU tensors, m = nu + nx.  F (batch, N, m, m), LN
    (batch, nx, nx) and info (batch, N + 1) int32 are written (allocated when
    None; F and LN zero-filled then, so their upper triangles read zero);
    ``work`` is a device tensor used as the workspace (allocated when None).
    Returns (F, LN, info)."""
    batch, N, m, nx = BAt.shape
    if m != nu + nx:
        raise ValueError("BAt rows must be nu + nx")
    if F is None:
        F = torch.zeros((batch, N, m, m), dtype=torch.float64, device=BAt.device).transpose(2, 3)
    if LN is None:
        LN = torch.zeros((batch, nx, nx), dtype=torch.float64, device=BAt.device).transpose(1, 2)
    if info is None:
        info = torch.empty((batch, N + 1), dtype=torch.int32, device=BAt.device)
    if work is None:
        work = riccati_workspace(nx, nu, batch, device=BAt.device)
    ldb, stb, sb = _stages(BAt, "BAt", m, nx)
    ldr, str_, sr = _stages(RSQ, "RSQ", m, m)
    ldf, stf, sf = _stages(F, "F", m, m)
    ldq, sq = _layout(QN, "QN", True)
    ldl, sl = _layout(LN, "LN", True)
    if info.dtype != torch.int32 or not info.is_contiguous() or info.numel() != batch * (N + 1):
        raise ValueError("info must be a contiguous int32 tensor of batch * (N + 1) entries")
    st = _lib.riccati_strided_batched(
        nx, nu, N, BAt.data_ptr(), ldb, stb, sb, RSQ.data_ptr(), ldr, str_, sr, QN.data_ptr(), ldq,
        sq, F.data_ptr(), ldf, stf, sf, LN.data_ptr(), ldl, sl, info.data_ptr(), work.data_ptr(),
        work.numel() * work.element_size(), batch, _stream(stream))
    _raise("mb_riccati_strided_batched", st)
    return F, LN, info


class Plan:
    """An uneven batch of dgemm / dpotrf problems run by one persistent kernel.

    ``problems`` is a sequence of dicts with the fields of struct mb_problem
    (device addresses as ints: A, B, C, info).  The plan records the
    addresses: the memory behind them must stay allocated while the plan
    lives.  ``execute`` enqueues on the current (or given) stream."""

    FUSED_GRAPH, FUSED, GROUPED, GROUPED_GRAPH = (_lib.PLAN_FUSED_GRAPH, _lib.PLAN_FUSED,
                                                  _lib.PLAN_GROUPED, _lib.PLAN_GROUPED_GRAPH)

    def __init__(self, problems, tile_two_min=None, potrf_waves=None):
        arr = problems if isinstance(problems, ctypes.Array) else _lib.problems_array(problems)
        st, self._h, bad = _lib.plan_create(arr, tile_two_min, potrf_waves)
        if st != _lib.MB_OK:
            raise MbError(f"mb_plan_create (problem {bad})", st)

    def execute(self, mode=None, stream=None):
        _raise("mb_plan_execute", _lib.plan_execute(self._h, _stream(stream), mode))

    def stats(self) -> dict:
        return _lib.plan_stats(self._h)

    def close(self):
        if self._h is not None:
            st = _lib.plan_destroy(self._h)
            self._h = None
            _raise("mb_plan_destroy", st)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        if getattr(self, "_h", None) is not None:
            _lib.plan_destroy(self._h)
            self._h = None
