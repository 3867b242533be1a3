"""Seeded synthetic inputs for the small-matrix FP64 dgemm / dpotrf workloads.

This module only draws numbers and lays them out; it contains none of the
routines' arithmetic and is shared, as the single source of inputs, by the
tests, the benchmark and the smoke check.  Both the HIP path and the CPU
oracle receive the very same bytes.

Workload shapes follow the paper's experimental setup: random square matrices
with n up to 300, sizes not known at compile time (Sec. 4); symmetric positive
definite inputs for the Cholesky factorization (Sec. 3.1.5, Sec. 5.2).

Layouts: a batch of column-major m x n matrices with leading dimension ld and
instance stride s is stored in one flat float64 buffer; instance b, element
(i, j) lives at offset b*s + i + j*ld.  ``colmajor`` returns that buffer as a
numpy array of shape (batch, cols, ld) in C order, so ``X[b].T[:rows]`` is the
matrix itself.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 190208115

# dgemm sweep: square m = n = k; batch per size such that A+B+C ~ 1 GiB.
GEMM_SWEEP_SIZES = (4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 300)
# dpotrf sweep: n, batch 4096 per size.
POTRF_SWEEP_SIZES = (8, 16, 32, 64, 128, 192, 256)
POTRF_SWEEP_BATCH = 4096
TRANS_CASES = ("NN", "NT", "TN", "TT")


def seed_for(config_index: int, size_index: int = 0) -> int:
    """Seed scheme: base + 1000*config + size index."""
    return SEED_BASE + 1000 * int(config_index) + int(size_index)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def gemm_sweep_batch(n: int) -> int:
    """Batch for square size n so that A, B and C together hold about 1 GiB."""
    return (1 << 30) // (24 * n * n)


def colmajor(g: np.random.Generator, batch: int, rows: int, cols: int, ld: int | None = None,
             pad_value: float = np.nan, low: float = -1.0, high: float = 1.0,
             integer: bool = False) -> np.ndarray:
    """Batch of column-major rows x cols matrices, uniform values in [low, high).

    Rows rows..ld-1 of every column are padding and hold ``pad_value`` (NaN by
    default, a sentinel that must survive untouched).  With ``integer`` the
    values are integers drawn uniformly from [low, high]."""
    ld = max(1, rows) if ld is None else ld
    if ld < max(1, rows):
        raise ValueError("ld must be >= max(1, rows)")
    out = np.full((batch, cols, ld), pad_value, dtype=np.float64)
    if integer:
        vals = g.integers(int(low), int(high) + 1, size=(batch, cols, rows)).astype(np.float64)
    else:
        vals = g.uniform(low, high, size=(batch, cols, rows))
    out[:, :, :rows] = vals
    return out


def matrix(X: np.ndarray, b: int, rows: int) -> np.ndarray:
    """View of instance b of a ``colmajor`` buffer as a rows x cols array."""
    return X[b].T[:rows]


def spd_batch(g: np.random.Generator, batch: int, n: int, ld: int | None = None,
              upper_value: float | None = None) -> np.ndarray:
    """A = M M^T + n I with M uniform in [-1, 1), exactly symmetric.

    Returned in the ``colmajor`` layout (batch, n, ld).  With ``upper_value``
    the strict upper triangle is overwritten by that value (a sentinel the
    lower-Cholesky routines must neither read nor write)."""
    ld = max(1, n) if ld is None else ld
    M = g.uniform(-1.0, 1.0, size=(batch, n, n))
    S = np.matmul(M, np.swapaxes(M, 1, 2))
    S = 0.5 * (S + np.swapaxes(S, 1, 2))
    S += n * np.eye(n)[None]
    out = np.full((batch, n, ld), np.nan, dtype=np.float64)
    # column-major: out[b, j, i] = A[i, j]; S is symmetric so S[b, j, i] works.
    out[:, :, :n] = S
    if upper_value is not None:
        iu = np.triu_indices(n, 1)  # (i < j) pairs -> element (i, j) lives at out[b, j, i]
        out[:, iu[1], iu[0]] = upper_value
    return out


def make_non_spd(g: np.random.Generator, A: np.ndarray, n: int):
    """Set one diagonal entry of one instance to -1.

    Returns (instance, column); the expected info of that instance is column+1
    for any correct lower Cholesky algorithm."""
    b = int(g.integers(0, A.shape[0]))
    j = int(g.integers(0, n))
    A[b, j, j] = -1.0
    return b, j


def log_uniform_sizes(g: np.random.Generator, count: int, lo: int, hi: int) -> np.ndarray:
    """Sizes floor(exp(U[ln lo, ln (hi+1)))) clipped to [lo, hi]."""
    s = np.floor(np.exp(g.uniform(math.log(lo), math.log(hi + 1), size=count))).astype(np.int64)
    return np.clip(s, lo, hi)


# ----------------------------------------------------------------------------
# Device-side generation (same recipes, drawn with torch's seeded generator
# directly in device memory; used where host generation of GiB-sized batches
# would dominate the run time).
# ----------------------------------------------------------------------------

def torch_colmajor(batch: int, rows: int, cols: int, ld: int | None = None, seed: int = 0,
                   device="cuda"):
    """Device tensor of shape (batch, rows, cols) with column-major strides
    (1 along rows, ld along cols, ld*cols between instances), uniform [-1, 1)."""
    import torch
    ld = max(1, rows) if ld is None else ld
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    base = torch.empty((batch, cols, ld), dtype=torch.float64, device=device)
    base.uniform_(-1.0, 1.0, generator=gen)
    return base.transpose(1, 2)[:, :rows, :]


def torch_spd(batch: int, n: int, seed: int = 0, device="cuda", chunk: int = 512):
    """Device tensor (batch, n, n), column-major, A = M M^T + n I, exactly symmetric."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    out = torch.empty((batch, n, n), dtype=torch.float64, device=device)
    eye = torch.eye(n, dtype=torch.float64, device=device)
    for b0 in range(0, batch, chunk):
        b1 = min(batch, b0 + chunk)
        M = torch.empty((b1 - b0, n, n), dtype=torch.float64, device=device)
        M.uniform_(-1.0, 1.0, generator=gen)
        S = torch.matmul(M, M.transpose(1, 2).contiguous())
        S = 0.5 * (S + S.transpose(1, 2))
        out[b0:b1] = S + n * eye
    # symmetric, so the row-major buffer is also the column-major one
    return out.transpose(1, 2)
