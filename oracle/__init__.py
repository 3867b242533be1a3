"""CPU oracle for the batched small-matrix FP64 dgemm / dpotrf('L') path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this package.  The product library
never loads it, and it shares no code with the HIP implementation.

The arithmetic lives in ``oracle.c`` (plain C, binary64, no fast-math, no FMA
contraction); this module only loads it with ctypes and marshals numpy arrays.
Each wrapper names the passage of Frison et al., "The BLAS API of BLASFEO:
optimizing performance for small matrices" (arXiv:1902.08115) it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# -ffp-contract=off: no fused multiply-add, every product is rounded as written.
# x86-64-v3 (AVX2) rather than -march=native: the library is built here and
# may run on a different host.
CFLAGS = ["-O2", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(src: str = _SRC, out: str = _LIB_PATH, extra_defines=()) -> str:
    """Compile oracle.c into a shared library with gcc and return its path."""
    cmd = ["gcc", *CFLAGS, *[f"-D{d}" for d in extra_defines], src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib = None


def load(path: str | None = None):
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or _LIB_PATH
    if not os.path.exists(p):
        build(out=p)
    lib = ctypes.CDLL(p)
    _declare(lib)
    if path is None:
        _lib = lib
    return lib


def _declare(lib):
    c_int, c_double, c_char, c_i64 = ctypes.c_int, ctypes.c_double, ctypes.c_char, ctypes.c_int64
    vp = ctypes.c_void_p
    lib.oracle_dgemm.argtypes = [c_char, c_char, c_int, c_int, c_int, c_double, vp, c_int,
                                 vp, c_int, c_double, vp, c_int]
    lib.oracle_dgemm.restype = None
    lib.oracle_dgemm_strided_batched.argtypes = [c_char, c_char, c_int, c_int, c_int, c_double,
                                                 vp, c_int, c_i64, vp, c_int, c_i64, c_double,
                                                 vp, c_int, c_i64, c_int, c_int]
    lib.oracle_dgemm_strided_batched.restype = None
    lib.oracle_dpotrf_l.argtypes = [c_int, vp, c_int]
    lib.oracle_dpotrf_l.restype = c_int
    lib.oracle_dpotrf_l_strided_batched.argtypes = [c_int, vp, c_int, c_i64, vp, c_int, c_int]
    lib.oracle_dpotrf_l_strided_batched.restype = None
    lib.oracle_dpotrf_l_adjoint.argtypes = [c_int, vp, c_int, vp, c_int, vp, c_int]
    lib.oracle_dpotrf_l_adjoint.restype = c_int
    lib.oracle_dpotrf_l_adjoint_strided_batched.argtypes = [c_int, vp, c_int, c_i64, vp, c_int,
                                                            c_i64, vp, c_int, c_i64, c_int, c_int]
    lib.oracle_dpotrf_l_adjoint_strided_batched.restype = c_int
    lib.oracle_dtrmm_rlnn.argtypes = [c_int, c_int, c_double, vp, c_int, vp, c_int]
    lib.oracle_dtrmm_rlnn.restype = None
    lib.oracle_dsyrk_ln.argtypes = [c_int, c_int, c_double, vp, c_int, c_double, vp, c_int]
    lib.oracle_dsyrk_ln.restype = None
    lib.oracle_riccati.argtypes = [c_int, c_int, c_int, vp, c_int, c_i64, vp, c_int, c_i64,
                                   vp, c_int, vp, c_int, c_i64, vp, c_int, vp]
    lib.oracle_riccati.restype = c_int
    lib.oracle_riccati_strided_batched.argtypes = [
        c_int, c_int, c_int, vp, c_int, c_i64, c_i64, vp, c_int, c_i64, c_i64, vp, c_int, c_i64,
        vp, c_int, c_i64, c_i64, vp, c_int, c_i64, vp, c_int, c_int]
    lib.oracle_riccati_strided_batched.restype = c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = c_int


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _check_f64(a: np.ndarray, name: str):
    if a.dtype != np.float64:
        raise TypeError(f"{name} must be float64")


def _storage(x: np.ndarray, name: str):
    """Return the leading dimension of a column-major 2-D float64 view.

    ``x`` may be a Fortran-ordered array, or a row slice ``X[:rows, :]`` of
    one (ld > rows); the oracle then sees the padded storage."""
    _check_f64(x, name)
    if x.ndim != 2:
        raise ValueError(f"{name} must be 2-D")
    s0, s1 = x.strides
    if x.shape[0] > 1 and x.shape[1] > 1 and s0 != 8:
        raise ValueError(f"{name} must be column-major (unit row stride)")
    ld = s1 // 8 if x.shape[1] > 1 else max(1, x.shape[0])
    return ld


def dgemm(transa: str, transb: str, alpha: float, A: np.ndarray, B: np.ndarray,
          beta: float, C: np.ndarray, k: int | None = None, lib=None) -> None:
    """C <= alpha*op(A)*op(B) + beta*C in place (Sec. 2.1 with the BLAS scalars).

    A, B, C are 2-D column-major float64 views (ld = column stride).  m, n are
    C's shape; k is read from op(A) unless given."""
    lib = lib or load()
    m, n = C.shape
    if k is None:
        k = A.shape[1] if transa in "Nn" else A.shape[0]
    lda, ldb, ldc = _storage(A, "A"), _storage(B, "B"), _storage(C, "C")
    lib.oracle_dgemm(transa.encode(), transb.encode(), m, n, k, float(alpha), _ptr(A), lda,
                     _ptr(B), ldb, float(beta), _ptr(C), ldc)


def dgemm_raw(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, lib=None):
    """Same operation on flat float64 buffers with explicit BLAS arguments."""
    lib = lib or load()
    for nm, a in (("A", A), ("B", B), ("C", C)):
        _check_f64(a, nm)
    lib.oracle_dgemm(transa.encode(), transb.encode(), m, n, k, float(alpha), _ptr(A), lda,
                     _ptr(B), ldb, float(beta), _ptr(C), ldc)


def dgemm_strided_batched(transa, transb, m, n, k, alpha, A, lda, strideA, B, ldb, strideB,
                          beta, C, ldc, strideC, batch, nthreads=0, lib=None):
    """Batched form on flat float64 buffers; instances are independent."""
    lib = lib or load()
    for nm, a in (("A", A), ("B", B), ("C", C)):
        _check_f64(a, nm)
    lib.oracle_dgemm_strided_batched(transa.encode(), transb.encode(), m, n, k, float(alpha),
                                     _ptr(A), lda, strideA, _ptr(B), ldb, strideB, float(beta),
                                     _ptr(C), ldc, strideC, batch, nthreads)


def dpotrf_l(A: np.ndarray, lib=None) -> int:
    """Lower Cholesky in place on a 2-D column-major view (Sec. 3.1.5); returns info."""
    lib = lib or load()
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    lda = _storage(A, "A")
    return int(lib.oracle_dpotrf_l(n, _ptr(A), lda))


def dpotrf_l_raw(n, A, lda, lib=None) -> int:
    lib = lib or load()
    _check_f64(A, "A")
    return int(lib.oracle_dpotrf_l(n, _ptr(A), lda))


def dpotrf_l_strided_batched(n, A, lda, strideA, batch, nthreads=0, lib=None) -> np.ndarray:
    lib = lib or load()
    _check_f64(A, "A")
    info = np.zeros(max(batch, 1), dtype=np.int32)
    lib.oracle_dpotrf_l_strided_batched(n, _ptr(A), lda, strideA, _ptr(info), batch, nthreads)
    return info[:batch]


def dpotrf_l_adjoint(L: np.ndarray, Lbar: np.ndarray, lib=None) -> np.ndarray:
    """Abar = sym(L^-T Phi(L^T tril(Lbar)) L^-1) for one n x n instance."""
    lib = lib or load()
    n = L.shape[0]
    Lf = np.asfortranarray(L, dtype=np.float64)
    Lb = np.asfortranarray(Lbar, dtype=np.float64)
    Ab = np.zeros((n, n), dtype=np.float64, order="F")
    rc = lib.oracle_dpotrf_l_adjoint(n, _ptr(Lf), max(n, 1), _ptr(Lb), max(n, 1), _ptr(Ab),
                                     max(n, 1))
    if rc != 0:
        raise MemoryError("oracle_dpotrf_l_adjoint: allocation failed")
    return Ab


def dpotrf_l_adjoint_strided_batched(n, L, ldl, strideL, Lbar, ldlb, strideLb, Abar, ldab,
                                     strideAb, batch, nthreads=0, lib=None):
    lib = lib or load()
    rc = lib.oracle_dpotrf_l_adjoint_strided_batched(n, _ptr(L), ldl, strideL, _ptr(Lbar), ldlb,
                                                     strideLb, _ptr(Abar), ldab, strideAb, batch,
                                                     nthreads)
    if rc != 0:
        raise MemoryError("oracle_dpotrf_l_adjoint_strided_batched: allocation failed")


def dtrmm_rlnn(alpha: float, A: np.ndarray, B: np.ndarray, lib=None) -> None:
    """B <= alpha * B * tril(A) in place (dtrmm 'R','L','N','N'; Sec. 3.1.4, Sec. 5.2)."""
    lib = lib or load()
    m, n = B.shape
    if A.shape[0] < n or A.shape[1] < n:
        raise ValueError("A must be at least n x n")
    lib.oracle_dtrmm_rlnn(m, n, float(alpha), _ptr(A), _storage(A, "A"), _ptr(B),
                          _storage(B, "B"))


def dsyrk_ln(alpha: float, A: np.ndarray, beta: float, C: np.ndarray, lib=None) -> None:
    """Lower triangle of C <= alpha * A * A^T + beta * C in place (dsyrk 'L','N';
    Sec. 3.1.2, Sec. 5.2)."""
    lib = lib or load()
    n, k = A.shape
    if C.shape != (n, n):
        raise ValueError("C must be n x n")
    lib.oracle_dsyrk_ln(n, k, float(alpha), _ptr(A), _storage(A, "A"), float(beta), _ptr(C),
                        _storage(C, "C"))


def riccati(BAt: np.ndarray, RSQ: np.ndarray, QN: np.ndarray, nu: int, lib=None):
    """Factorized backward Riccati recursion of Sec. 5.2 for one problem.

    BAt: (N, m, nx) stage matrices [B^T; A^T]; RSQ: (N, m, m) stage matrices
    [R S; S^T Q] (lower triangle read); QN: (nx, nx).  Returns (F, LN, info)
    with F (N, m, m) the stage factors (lower triangles written, the rest
    zero), LN = chol(QN) and info (N + 1,) as documented in oracle.c."""
    lib = lib or load()
    N, m, nx = BAt.shape
    if m != nu + nx or RSQ.shape != (N, m, m) or QN.shape != (nx, nx):
        raise ValueError("inconsistent Riccati shapes")
    # column-major stage matrices: element (i, j) of stage n at n*m*c + j*m + i
    bat = np.ascontiguousarray(np.swapaxes(BAt, 1, 2), dtype=np.float64)
    rsq = np.ascontiguousarray(np.swapaxes(RSQ, 1, 2), dtype=np.float64)
    q = np.asfortranarray(QN, dtype=np.float64)
    F = np.zeros((max(N, 1), m, m), dtype=np.float64)
    LN = np.zeros((nx, nx), dtype=np.float64, order="F")
    info = np.zeros(N + 1, dtype=np.int32)
    rc = lib.oracle_riccati(nx, nu, N, _ptr(bat), max(m, 1), m * nx, _ptr(rsq), max(m, 1), m * m,
                            _ptr(q), max(nx, 1), _ptr(F), max(m, 1), m * m, _ptr(LN), max(nx, 1),
                            _ptr(info))
    if rc != 0:
        raise MemoryError("oracle_riccati: allocation failed")
    return np.swapaxes(F[:N], 1, 2).copy(), np.array(LN), info


def riccati_strided_batched(nx, nu, N, BAt, ldbat, sbat, strideBAt, RSQ, ldrsq, srsq, strideRSQ,
                            QN, ldq, strideQ, F, ldf, sf, strideF, LN, ldl, strideL, info, batch,
                            nthreads=0, lib=None):
    """Batched form on flat buffers (stage stride s*, problem stride stride*)."""
    lib = lib or load()
    for nm, a in (("BAt", BAt), ("RSQ", RSQ), ("QN", QN), ("F", F), ("LN", LN)):
        _check_f64(a, nm)
    if info.dtype != np.int32:
        raise TypeError("info must be int32")
    rc = lib.oracle_riccati_strided_batched(nx, nu, N, _ptr(BAt), ldbat, sbat, strideBAt,
                                            _ptr(RSQ), ldrsq, srsq, strideRSQ, _ptr(QN), ldq,
                                            strideQ, _ptr(F), ldf, sf, strideF, _ptr(LN), ldl,
                                            strideL, _ptr(info), batch, nthreads)
    if rc != 0:
        raise MemoryError("oracle_riccati_strided_batched: allocation failed")


def num_threads(lib=None) -> int:
    return int((lib or load()).oracle_num_threads())
