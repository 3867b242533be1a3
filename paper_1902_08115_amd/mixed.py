"""C_b = chol(A_b) B_b, and its reverse-mode derivative, over a batch whose
instances have different orders n_b (B_b is n_b x nb): each phase is one
fused plan (one persistent kernel launch through a HIP graph).

  forward:   L = A (copy), L = chol(L) [plan], strict upper of L = 0 [plan],
             C = L B [plan]
  backward:  Bbar = L^T Cbar and Lbar = Cbar B^T [one plan, 2 problems per
             instance], Abar = Cholesky adjoint(L, Lbar) [plan]

Every operand lives in one flat FP64 device arena per role, instance after
instance, tight leading dimensions; ``view(role, b)`` returns instance b as a
(rows, cols) column-major view.

Calling the object, ``C = mp(A, B)`` with A and B flat arenas of that layout,
runs the forward through a ``torch.autograd.Function``; ``C.backward(Cbar)``
(or any loss built on C) then runs the backward plans, and A.grad, B.grad
receive Abar and Bbar.  C is a view of the object's own C arena, as the
output of a captured graph is: the next forward overwrites it, and a
backward whose forward has been overwritten raises.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib, blas


class MixedCholeskyProduct:
    ROLES = ("A", "B", "L", "C", "Cbar", "Lbar", "Bbar", "Abar")

    def __init__(self, ns, nb: int, device="cuda"):
        self.ns = np.asarray(ns, dtype=np.int64)
        self.nb = int(nb)
        self.count = len(self.ns)
        sq = self.ns * self.ns
        rect = self.ns * self.nb
        self.off_sq = np.concatenate([[0], np.cumsum(sq)[:-1]]).astype(np.int64)
        self.off_rect = np.concatenate([[0], np.cumsum(rect)[:-1]]).astype(np.int64)
        nsq, nrect = int(sq.sum()), int(rect.sum())
        self.buf = {}
        for r in self.ROLES:
            size = nsq if r in ("A", "L", "Lbar", "Abar") else nrect
            self.buf[r] = torch.zeros(max(size, 1), dtype=torch.float64, device=device)
        self.info = torch.zeros(max(self.count, 1), dtype=torch.int32, device=device)
        ptr = {r: t.data_ptr() for r, t in self.buf.items()}
        sqp = lambda r, i: ptr[r] + 8 * int(self.off_sq[i])  # noqa: E731
        rcp = lambda r, i: ptr[r] + 8 * int(self.off_rect[i])  # noqa: E731
        P = []  # (name, problems)
        potrf, laset, gemm, gemm_b, adj = [], [], [], [], []
        for i, n in enumerate(self.ns.tolist()):
            potrf.append(dict(op=_lib.OP_DPOTRF, uplo="L", n=n, ldc=n, C=sqp("L", i),
                              info=self.info.data_ptr() + 4 * i))
            if n > 1:
                laset.append(dict(op=_lib.OP_DLASET, uplo="U", m=n - 1, n=n - 1, alpha=0.0,
                                  beta=0.0, ldc=n, C=sqp("L", i) + 8 * n))
            gemm.append(dict(op=_lib.OP_DGEMM, transa="N", transb="N", m=n, n=self.nb, k=n,
                             alpha=1.0, beta=0.0, A=sqp("L", i), lda=n, B=rcp("B", i), ldb=n,
                             C=rcp("C", i), ldc=n))
            gemm_b.append(dict(op=_lib.OP_DGEMM, transa="T", transb="N", m=n, n=self.nb, k=n,
                               alpha=1.0, beta=0.0, A=sqp("L", i), lda=n, B=rcp("Cbar", i),
                               ldb=n, C=rcp("Bbar", i), ldc=n))
            gemm_b.append(dict(op=_lib.OP_DGEMM, transa="N", transb="T", m=n, n=n, k=self.nb,
                               alpha=1.0, beta=0.0, A=rcp("Cbar", i), lda=n, B=rcp("B", i),
                               ldb=n, C=sqp("Lbar", i), ldc=n))
            adj.append(dict(op=_lib.OP_DPOTRF_ADJOINT, n=n, A=sqp("L", i), lda=n,
                            B=sqp("Lbar", i), ldb=n, C=sqp("Abar", i), ldc=n))
        self.plans = {name: blas.Plan(pr) for name, pr in (("potrf", potrf), ("laset", laset),
                                                           ("gemm", gemm), ("gemm_b", gemm_b),
                                                           ("adjoint", adj))}
        self.forwards = 0  # forward count: a backward must follow its own forward

    def __call__(self, A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
        """C = chol(A) B for flat arenas A (sum n_b^2) and B (sum n_b nb),
        differentiable in both (symmetric gradient for A)."""
        return _MixedCholeskyProductFn.apply(A, B, self)

    def load(self, role: str, X: torch.Tensor):
        """Copy X into the role's arena (nothing to do if X is the arena)."""
        dst = self.buf[role]
        if X.dtype != torch.float64 or X.device != dst.device or X.numel() != dst.numel():
            raise ValueError(f"{role}: expected {dst.numel()} float64 values on {dst.device}")
        if X.data_ptr() != dst.data_ptr():
            dst.copy_(X.reshape(-1))

    def symmetrize_index(self) -> torch.Tensor:
        """Index t with X[t] = instance-wise transpose of the A-shaped arena X."""
        parts = []
        for b, n in enumerate(self.ns.tolist()):
            j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")  # element i + j n
            parts.append(int(self.off_sq[b]) + (j + i * n).ravel())
        idx = np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)
        return torch.from_numpy(idx.astype(np.int64)).to(self.buf["A"].device)

    def view(self, role: str, b: int) -> torch.Tensor:
        n = int(self.ns[b])
        if role in ("A", "L", "Lbar", "Abar"):
            o, cols = int(self.off_sq[b]), n
        else:
            o, cols = int(self.off_rect[b]), self.nb
        return self.buf[role][o:o + n * cols].view(cols, n).t()

    def forward(self, mode=None, stream=None):
        self.buf["L"].copy_(self.buf["A"])
        for name in ("potrf", "laset", "gemm"):
            self.plans[name].execute(mode, stream)
        self.forwards += 1

    def backward(self, mode=None, stream=None):
        for name in ("gemm_b", "adjoint"):
            self.plans[name].execute(mode, stream)

    def close(self):
        for p in self.plans.values():
            p.close()
        self.plans = {}


class _MixedCholeskyProductFn(torch.autograd.Function):
    """Forward and backward plans of a MixedCholeskyProduct behind autograd."""

    @staticmethod
    def forward(ctx, A, B, mp):
        mp.load("A", A)
        mp.load("B", B)
        mp.forward()
        ctx.mp, ctx.version = mp, mp.forwards
        return mp.buf["C"].view(-1)

    @staticmethod
    def backward(ctx, Cbar):
        mp = ctx.mp
        if mp.forwards != ctx.version:
            raise RuntimeError("MixedCholeskyProduct: a later forward overwrote the factors "
                               "this backward needs")
        mp.load("Cbar", Cbar.contiguous())
        mp.backward()
        gA = mp.buf["Abar"].clone() if ctx.needs_input_grad[0] else None
        gB = mp.buf["Bbar"].clone() if ctx.needs_input_grad[1] else None
        return gA, gB, None
