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


# ----------------------------------------------------------------------------
# Uneven batch: independent dgemm and dpotrf problems of mixed sizes.
# ----------------------------------------------------------------------------

UNEVEN_COUNT = 100_000
UNEVEN_LO, UNEVEN_HI = 4, 160
UNEVEN_P_GEMM = 0.7


def uneven_spec(count: int, seed: int, lo: int = UNEVEN_LO, hi: int = UNEVEN_HI,
                p_gemm: float = UNEVEN_P_GEMM, non_spd_frac: float = 0.0) -> dict:
    """Problem list of an uneven batch.

    Each problem is a dgemm with probability p_gemm, else a lower dpotrf.  m,
    n, k are independent log-uniform draws in [lo, hi] (a dpotrf uses n as its
    order); transa, transb are 'N'/'T' with probability 1/2 each; alpha =
    beta = 1.  A fraction non_spd_frac of the dpotrf problems gets one
    diagonal entry -1 at a seeded column (fail_col >= 0, expected info
    fail_col + 1); the others have fail_col = -1.

    Every operand is stored tight (ld = rows) in one arena, problem after
    problem: dgemm A, B, C; dpotrf its n x n matrix (at off_c).  Returns numpy
    arrays op (0 dgemm, 1 dpotrf), ta, tb, m, n, k, lda, ldb, ldc, off_a,
    off_b, off_c, fail_col and the arena length `total` (elements)."""
    g = rng(seed)
    op = (g.uniform(size=count) >= p_gemm).astype(np.int64)
    m = log_uniform_sizes(g, count, lo, hi)
    n = log_uniform_sizes(g, count, lo, hi)
    k = log_uniform_sizes(g, count, lo, hi)
    ta = g.integers(0, 2, size=count)
    tb = g.integers(0, 2, size=count)
    fail_draw = g.uniform(size=count)
    fail_pos = g.uniform(size=count)
    gemm = op == 0
    lda = np.where(gemm, np.where(ta == 0, m, k), 0)
    acols = np.where(gemm, np.where(ta == 0, k, m), 0)
    ldb = np.where(gemm, np.where(tb == 0, k, n), 0)
    bcols = np.where(gemm, np.where(tb == 0, n, k), 0)
    ldc = np.where(gemm, m, n)
    size_a = lda * acols
    size_b = ldb * bcols
    size_c = ldc * n
    ends = np.cumsum(size_a + size_b + size_c)
    start = ends - (size_a + size_b + size_c)
    fail_col = np.where((~gemm) & (fail_draw < non_spd_frac),
                        np.minimum((fail_pos * n).astype(np.int64), n - 1), -1)
    return dict(op=op, ta=ta, tb=tb, m=m, n=n, k=k, lda=lda, ldb=ldb, ldc=ldc,
                off_a=start, off_b=start + size_a, off_c=start + size_a + size_b,
                fail_col=fail_col, total=int(ends[-1]) if count else 0, count=count,
                alpha=1.0, beta=1.0)


def uneven_host(spec: dict, seed: int) -> np.ndarray:
    """Host arena for ``spec``: uniform [-1, 1) everywhere, then every dpotrf
    matrix replaced by M M^T + n I (exactly symmetric) and its fail column set."""
    g = rng(seed)
    X = g.uniform(-1.0, 1.0, size=spec["total"])
    for i in np.nonzero(spec["op"] == 1)[0]:
        n = int(spec["n"][i])
        S = spd_batch(g, 1, n)[0]  # (n, n) column-major, ld = n
        o = int(spec["off_c"][i])
        X[o:o + n * n] = S.ravel()
        f = int(spec["fail_col"][i])
        if f >= 0:
            X[o + f + f * n] = -1.0
    return X


def uneven_device(spec: dict, seed: int, device="cuda"):
    """Device arena for ``spec`` drawn with torch's seeded generator (the same
    recipe as ``uneven_host``, different random stream): one flat float64
    tensor."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    X = torch.empty(spec["total"], dtype=torch.float64, device=device)
    X.uniform_(-1.0, 1.0, generator=gen)
    pot = np.nonzero(spec["op"] == 1)[0]
    sizes = spec["n"][pot]
    for si, n in enumerate(np.unique(sizes)):
        n = int(n)
        idx = pot[sizes == n]
        S = torch_spd(len(idx), n, seed=int(seed) * 1000 + si, device=device)
        S = S.transpose(1, 2).reshape(len(idx), n * n)  # symmetric: same bytes either way
        offs = torch.as_tensor(spec["off_c"][idx], dtype=torch.int64, device=device)
        flat = (offs[:, None] + torch.arange(n * n, device=device)[None, :]).reshape(-1)
        X.index_copy_(0, flat, S.reshape(-1))
    fail = np.nonzero(spec["fail_col"] >= 0)[0]
    if len(fail):
        f = spec["fail_col"][fail]
        pos = spec["off_c"][fail] + f + f * spec["n"][fail]
        X[torch.as_tensor(pos, dtype=torch.int64, device=device)] = -1.0
    return X


# ----------------------------------------------------------------------------
# Differentiation workload: C = chol(A) B with B n x 32.
# ----------------------------------------------------------------------------

BACKWARD_BATCH = 8192
BACKWARD_N = 64
BACKWARD_NB = 32
BACKWARD_MIXED_COUNT = 2048
BACKWARD_MIXED_LO, BACKWARD_MIXED_HI = 16, 192
FD_DIRECTIONS = 50
FD_STEP = 1e-6


def backward_mixed_sizes(seed: int, count: int = BACKWARD_MIXED_COUNT) -> np.ndarray:
    """Orders n = floor(exp(U[ln 16, ln 193))) of the mixed differentiation batch."""
    return log_uniform_sizes(rng(seed), count, BACKWARD_MIXED_LO, BACKWARD_MIXED_HI)


def torch_symmetric(batch: int, n: int, seed: int, device="cuda"):
    """Device tensor (batch, n, n), column-major, symmetric with entries
    (X + X^T)/2 of X uniform [-1, 1) (finite-difference directions)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    X = torch.empty((batch, n, n), dtype=torch.float64, device=device)
    X.uniform_(-1.0, 1.0, generator=gen)
    X = 0.5 * (X + X.transpose(1, 2))
    return X.contiguous().transpose(1, 2)


# ----------------------------------------------------------------------------
# Riccati recursion (Sec. 5.2): horizon N = 10, (nx, nu) of the paper's
# Table 2.  The paper does not give its system matrices; the recipe below
# draws well-conditioned ones: BAt_n = [B_n^T; A_n^T] uniform [-1, 1) / sqrt(nx)
# (spectral radius of A about 1, so P_n neither explodes nor vanishes over the
# horizon), RSQ_n = W W^T / m + I and Q_N = V V^T / nx + I with W, V uniform
# [-1, 1) (symmetric positive definite, eigenvalues in [1, 1 + m/3]).
# ----------------------------------------------------------------------------

RICCATI_N = 10
RICCATI_SHAPES = ((8, 4), (24, 12), (40, 20), (64, 32))
# problems per batch: enough waves to fill the device several times over for
# every shape, about 4-16 GB of operands per shape
RICCATI_BATCH = {(8, 4): 131072, (24, 12): 32768, (40, 20): 16384, (64, 32): 8192}


def torch_riccati(nx: int, nu: int, N: int, batch: int, seed: int, device="cuda",
                  chunk: int = 1024):
    """(BAt, RSQ, QN): column-major FP64 tensors of shapes (batch, N, m, nx),
    (batch, N, m, m) and (batch, nx, nx), m = nu + nx, drawn by the recipe
    above with one seeded generator (BAt first, then RSQ, then QN, in chunks
    of `chunk` problems)."""
    import torch
    m = nu + nx
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    f64 = torch.float64
    bat = torch.empty((batch, N, nx, m), dtype=f64, device=device)
    rsq = torch.empty((batch, N, m, m), dtype=f64, device=device)
    q = torch.empty((batch, nx, nx), dtype=f64, device=device)
    eye_m = torch.eye(m, dtype=f64, device=device)
    eye_x = torch.eye(nx, dtype=f64, device=device)
    for b0 in range(0, batch, chunk):
        b1 = min(batch, b0 + chunk)
        bat[b0:b1].uniform_(-1.0, 1.0, generator=gen)
        bat[b0:b1] *= 1.0 / math.sqrt(max(nx, 1))
        W = torch.empty((b1 - b0, N, m, m), dtype=f64, device=device)
        W.uniform_(-1.0, 1.0, generator=gen)
        S = torch.matmul(W, W.transpose(2, 3).contiguous()) / max(m, 1)
        rsq[b0:b1] = 0.5 * (S + S.transpose(2, 3)) + eye_m
        V = torch.empty((b1 - b0, nx, nx), dtype=f64, device=device)
        V.uniform_(-1.0, 1.0, generator=gen)
        T = torch.matmul(V, V.transpose(1, 2).contiguous()) / max(nx, 1)
        q[b0:b1] = 0.5 * (T + T.transpose(1, 2)) + eye_x
    # RSQ and QN are symmetric: their row-major buffers are the column-major ones
    return bat.transpose(2, 3), rsq.transpose(2, 3), q.transpose(1, 2)

