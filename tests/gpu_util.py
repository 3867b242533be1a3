"""Helpers for the GPU parity tests: device buffers from the seeded inputs,
calls through the C ABI, and comparisons against the CPU oracle."""
from __future__ import annotations

import sys

import numpy as np

import oracle
from paper_1902_08115_amd import inputs

# Parity gates: normwise relative error of dgemm and Cholesky reconstruction
# residual, both 1e-12 (FP64 throughout; the expected error is ~1e-16..1e-15).
GEMM_TOL = 1e-12
POTRF_TOL = 1e-12


def say(msg: str):
    """Name the case before a GPU step (flushed, so a fault still leaves it)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def torch_mods():
    import torch

    from paper_1902_08115_amd import _lib, blas  # raises loudly if the library is missing
    return torch, _lib, blas


def dev(X: np.ndarray):
    """Host (batch, cols, ld) buffer -> flat device tensor holding the same bytes."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(X).ravel()).cuda()


def host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gemm_dims(ta: str, tb: str, m: int, n: int, k: int):
    """(rows, cols) of the stored A and B."""
    a = (m, k) if ta == "N" else (k, m)
    b = (k, n) if tb == "N" else (n, k)
    return a, b


def oracle_gemm_batch(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, batch):
    """Oracle over a (batch, cols, ld) host batch; returns the new C buffer."""
    Cr = np.ascontiguousarray(C).ravel().copy()
    sA = A.shape[1] * A.shape[2]
    sB = B.shape[1] * B.shape[2]
    sC = C.shape[1] * C.shape[2]
    oracle.dgemm_strided_batched(ta, tb, m, n, k, alpha, np.ascontiguousarray(A).ravel(), lda, sA,
                                 np.ascontiguousarray(B).ravel(), ldb, sB, beta, Cr, ldc, sC,
                                 batch, nthreads=0)
    return Cr.reshape(C.shape)


def gemm_errors(Cg, Cr, A, B, C0, ta, tb, m, n, k, alpha, beta):
    """Per-instance max of the two normwise relative errors (plain and scaled)."""
    e1 = e2 = 0.0
    for b in range(Cg.shape[0]):
        g = Cg[b].T[:m, :n]
        r = Cr[b].T[:m, :n]
        d = np.linalg.norm(g - r)
        nr = np.linalg.norm(r)
        e1 = max(e1, d / nr if nr > 0 else d)
        Am = A[b].T[:(m if ta == "N" else k), :(k if ta == "N" else m)]
        Bm = B[b].T[:(k if tb == "N" else n), :(n if tb == "N" else k)]
        scale = abs(alpha) * np.linalg.norm(Am) * np.linalg.norm(Bm) + abs(beta) * np.linalg.norm(
            C0[b].T[:m, :n])
        e2 = max(e2, d / scale if scale > 0 else d)
    return e1, e2


def potrf_check(Ag, Aref_in, n, lda):
    """Per-instance (residual, L-vs-oracle error) maxima and info from the oracle."""
    batch = Ag.shape[0]
    X = np.ascontiguousarray(Aref_in).ravel().copy()
    info = oracle.dpotrf_l_strided_batched(n, X, lda, Aref_in.shape[1] * Aref_in.shape[2], batch)
    Lr_all = X.reshape(Aref_in.shape)
    res = lerr = 0.0
    for b in range(batch):
        if info[b] != 0:
            continue
        A0 = Aref_in[b].T[:n, :n]
        A0 = np.tril(A0) + np.tril(A0, -1).T
        Lg = np.tril(Ag[b].T[:n, :n])
        Lr = np.tril(Lr_all[b].T[:n, :n])
        Ll = Lg.astype(np.longdouble)
        r = np.sqrt(((A0.astype(np.longdouble) - Ll @ Ll.T) ** 2).sum()) / np.sqrt(
            (A0.astype(np.longdouble) ** 2).sum())
        res = max(res, float(r))
        lerr = max(lerr, np.linalg.norm(Lg - Lr) / np.linalg.norm(Lr))
    return res, lerr, info, Lr_all


__all__ = ["inputs"]
