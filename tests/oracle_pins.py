"""Pins that tie the CPU oracle to facts fixed outside it.

Every check takes the ctypes handle of an oracle build, so the same checks run
against the real oracle (tests/test_oracle_pins.py) and against deliberately
broken copies of it (tests/test_oracle_mutants.py), which must each fail at
least one of them.

What pins what (all CPU, no GPU):
  * exact rational brute force on tiny dgemm shapes, all trans cases, ld
    padding with NaN sentinels (integer data: the exact result is a binary64
    number, so the oracle must return it bit for bit);
  * dgemm closed forms: identity, permutation, all-ones, single non-zero;
  * the transposition rule (A B)^T = B^T A^T (paper Sec. 2.2, variant 'D', TT);
  * SciPy/OpenBLAS dgemm and LAPACK dpotrf as independent libraries;
  * dpotrf: the info closed form, exact integer factors, identity/diagonal,
    the Pascal and 3x3 textbook fixtures, the 1x1/2x2 closed forms, the
    reconstruction residual, untouched upper triangle;
  * Cholesky adjoint: log-det closed form (Abar = A^-1), n = 1, central finite
    differences;
  * dtrmm_rlnn / dsyrk_ln: exact rational brute force with NaN sentinels in
    the parts that must not be read or written, SciPy/OpenBLAS dtrmm and dsyrk;
  * Riccati recursion: the closed-form update of Sec. 5.2 (solved with a
    general linear solve, not a Cholesky factorization), the scalar closed
    form, convergence to SciPy's discrete algebraic Riccati solution on a long
    horizon, the info and not-computed-stage rules, batched == single.
"""
from __future__ import annotations

import itertools
import math
import os
from fractions import Fraction

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TRANS = ("N", "T")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _colmajor_padded(g, rows, cols, pad, integer=True, lo=-4, hi=4):
    ld = max(1, rows + pad)
    X = np.full((ld, max(cols, 1)), np.nan, order="F")
    if integer:
        X[:rows, :cols] = g.integers(lo, hi + 1, size=(rows, cols))
    else:
        X[:rows, :cols] = g.uniform(-1, 1, size=(rows, cols))
    return X, ld


def _op(X, t, rows, cols):
    """Rows x cols matrix op(X) as a Python list of lists (exact values)."""
    if t == "N":
        return [[X[i, j] for j in range(cols)] for i in range(rows)]
    return [[X[j, i] for j in range(cols)] for i in range(rows)]


def _load_pair(name):
    rows, mats, cur = [], [], []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line.startswith("#"):
                if cur:
                    mats.append(np.array(cur, dtype=np.float64))
                    cur = []
                continue
            if line:
                cur.append([float(v) for v in line.split()])
    if cur:
        mats.append(np.array(cur, dtype=np.float64))
    return mats[0], mats[1]


# ----------------------------------------------------------------------------
# dgemm
# ----------------------------------------------------------------------------

def pin_dgemm_exact_bruteforce(lib, sizes=range(0, 6), pads=(0, 3), seed=11):
    """Exhaustive m, n, k in 0..5, four trans cases, ld padding 0 and 3.

    Integer entries in [-4, 4], alpha and beta in {0, +-1, +-2, +-0.5}: the
    exact rational result (Fractions) is representable in binary64, so the
    oracle must reproduce it exactly; NaN sentinels in the padding rows of C
    must be untouched, and NaN padding of A and B must never be read."""
    g = _rng(seed)
    scal = [0.0, 1.0, -1.0, 2.0, -2.0, 0.5, -0.5]
    for m, n, k in itertools.product(sizes, sizes, sizes):
        for ta, tb in itertools.product(TRANS, TRANS):
            pad = pads[(m + n + k) % len(pads)]
            ar, ac = (m, k) if ta == "N" else (k, m)
            br, bc = (k, n) if tb == "N" else (n, k)
            A, lda = _colmajor_padded(g, ar, ac, pad)
            B, ldb = _colmajor_padded(g, br, bc, pad)
            C, ldc = _colmajor_padded(g, m, n, pad)
            alpha = scal[int(g.integers(len(scal)))]
            beta = scal[int(g.integers(len(scal)))]
            opA, opB = _op(A, ta, m, k), _op(B, tb, k, n)
            exp = C.copy()
            quick = (alpha == 0.0 or k == 0) and beta == 1.0
            for i in range(m):
                for j in range(n):
                    if quick:
                        continue
                    s = sum((Fraction(opA[i][p]) * Fraction(opB[p][j]) for p in range(k)),
                            Fraction(0))
                    v = Fraction(alpha) * s
                    if beta != 0.0:
                        v += Fraction(beta) * Fraction(C[i, j])
                    exp[i, j] = float(v)
            got = C.copy(order="F")
            oracle.dgemm_raw(ta, tb, m, n, k, alpha, A.ravel(order="F"), lda,
                             B.ravel(order="F"), ldb, beta, got_flat := got.ravel(order="F"),
                             ldc, lib=lib)
            got = got_flat.reshape(got.shape, order="F")
            ok = np.array_equal(got, exp, equal_nan=True)
            assert ok, f"exact mismatch m={m} n={n} k={k} {ta}{tb} alpha={alpha} beta={beta}"


def pin_dgemm_lowercase_and_conj_flags(lib, seed=12):
    """'n'/'t'/'c'/'C' behave as 'N'/'T'/'T'/'T' for real data."""
    g = _rng(seed)
    m, n, k = 5, 4, 3
    for up, variants in (("N", "n"), ("T", "tcC")):
        for low in variants:
            ar, ac = (m, k) if up == "N" else (k, m)
            A, lda = _colmajor_padded(g, ar, ac, 0)
            B, ldb = _colmajor_padded(g, k, n, 0)
            C0, ldc = _colmajor_padded(g, m, n, 0)
            c1, c2 = C0.ravel(order="F").copy(), C0.ravel(order="F").copy()
            oracle.dgemm_raw(up, "N", m, n, k, 1.0, A.ravel(order="F"), lda, B.ravel(order="F"),
                             ldb, 1.0, c1, ldc, lib=lib)
            oracle.dgemm_raw(low, "n", m, n, k, 1.0, A.ravel(order="F"), lda, B.ravel(order="F"),
                             ldb, 1.0, c2, ldc, lib=lib)
            assert np.array_equal(c1, c2), f"flag {low!r} differs from {up!r}"


def pin_dgemm_closed_forms(lib, seed=13):
    """Identity, permutation, all-ones and single non-zero factors."""
    g = _rng(seed)
    m = n = k = 7
    for ta, tb in itertools.product(TRANS, TRANS):
        # identity left factor: C = alpha*op(B) + beta*C, exact for alpha, beta powers of two
        B, ldb = _colmajor_padded(g, k if tb == "N" else n, n if tb == "N" else k, 2,
                                  integer=False)
        C, ldc = _colmajor_padded(g, m, n, 1, integer=False)
        I = np.asfortranarray(np.eye(m))
        got = C.copy(order="F")
        oracle.dgemm(ta, tb, 2.0, I, B[: (k if tb == "N" else n)], 0.5, got[:m], lib=lib)
        opB = B[:k, :n] if tb == "N" else B[:n, :k].T
        assert np.array_equal(got[:m, :n], 2.0 * opB + 0.5 * C[:m, :n]), f"identity {ta}{tb}"
        assert np.isnan(got[m:]).all(), "padding rows touched"
        # permutation: op(A) = P permutes the rows of op(B) exactly
        perm = g.permutation(m)
        P = np.zeros((m, k))
        P[np.arange(m), perm] = 1.0
        Ast = np.asfortranarray(P if ta == "N" else P.T)
        got = np.zeros((m, n), order="F")
        oracle.dgemm(ta, tb, 1.0, Ast, B[: (k if tb == "N" else n)], 0.0, got, lib=lib)
        assert np.array_equal(got, opB[perm, :]), f"permutation {ta}{tb}"
        # all-ones: every entry equals alpha*k + beta*c0
        ones_a = np.ones((m, k) if ta == "N" else (k, m), order="F")
        ones_b = np.ones((k, n) if tb == "N" else (n, k), order="F")
        C0 = np.asfortranarray(g.integers(-4, 5, size=(m, n)).astype(np.float64))
        got = C0.copy(order="F")
        oracle.dgemm(ta, tb, -2.0, ones_a, ones_b, 3.0, got, lib=lib)
        assert np.array_equal(got, -2.0 * k + 3.0 * C0), f"all-ones {ta}{tb}"
        # single non-zero op(A) = e_i e_p^T selects row p of op(B) into row i
        i0, p0 = 2, 5
        E = np.zeros((m, k))
        E[i0, p0] = 1.0
        Est = np.asfortranarray(E if ta == "N" else E.T)
        got = np.zeros((m, n), order="F")
        oracle.dgemm(ta, tb, 1.0, Est, B[: (k if tb == "N" else n)], 0.0, got, lib=lib)
        expct = np.zeros((m, n))
        expct[i0] = opB[p0]
        assert np.array_equal(got, expct), f"single non-zero {ta}{tb}"


def pin_dgemm_transposition_rule(lib, seed=14):
    """dgemm(T,T,A,B) equals (dgemm(N,N,B,A))^T bit for bit on integer data
    (the transposition rule used for the 'TT' kernel of variant 'D', Sec. 2.2)."""
    g = _rng(seed)
    for m, n, k in [(3, 5, 4), (8, 2, 9), (1, 6, 1)]:
        A = np.asfortranarray(g.integers(-4, 5, size=(k, m)).astype(np.float64))  # op(A) = A^T
        B = np.asfortranarray(g.integers(-4, 5, size=(n, k)).astype(np.float64))  # op(B) = B^T
        C1 = np.zeros((m, n), order="F")
        oracle.dgemm("T", "T", 1.0, A, B, 0.0, C1, lib=lib)
        C2 = np.zeros((n, m), order="F")
        oracle.dgemm("N", "N", 1.0, B, A, 0.0, C2, lib=lib)
        assert np.array_equal(C1, C2.T)


def pin_dgemm_scipy(lib, seed=15):
    """Random U[-1,1) data against SciPy's dgemm (OpenBLAS), all trans cases."""
    from scipy.linalg import blas
    g = _rng(seed)
    for m, n, k in [(17, 9, 33), (32, 32, 32), (5, 40, 3), (64, 48, 80)]:
        for ta, tb in itertools.product(TRANS, TRANS):
            A = np.asfortranarray(g.uniform(-1, 1, size=(m, k) if ta == "N" else (k, m)))
            B = np.asfortranarray(g.uniform(-1, 1, size=(k, n) if tb == "N" else (n, k)))
            C = np.asfortranarray(g.uniform(-1, 1, size=(m, n)))
            ref = blas.dgemm(0.75, A, B, beta=-1.25, c=C.copy(order="F"),
                             trans_a=int(ta == "T"), trans_b=int(tb == "T"))
            got = C.copy(order="F")
            oracle.dgemm(ta, tb, 0.75, A, B, -1.25, got, lib=lib)
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            assert err <= 1e-14, f"scipy mismatch {ta}{tb} {m}x{n}x{k}: {err}"


def pin_dgemm_special_scalars(lib, seed=16):
    """beta = 0 never reads C (NaN in C does not propagate); alpha = 0 and
    k = 0 never read A, B; quick return with beta = 1 leaves C untouched."""
    g = _rng(seed)
    m, n, k = 4, 3, 5
    A = np.asfortranarray(g.uniform(-1, 1, size=(m, k)))
    B = np.asfortranarray(g.uniform(-1, 1, size=(k, n)))
    C = np.full((m, n), np.nan, order="F")
    oracle.dgemm("N", "N", 1.0, A, B, 0.0, C, lib=lib)
    assert np.isfinite(C).all(), "beta = 0 must not read C"
    An = np.full((m, k), np.nan, order="F")
    Bn = np.full((k, n), np.nan, order="F")
    C0 = np.asfortranarray(g.uniform(-1, 1, size=(m, n)))
    C = C0.copy(order="F")
    oracle.dgemm("N", "N", 0.0, An, Bn, 2.0, C, lib=lib)
    assert np.array_equal(C, 2.0 * C0), "alpha = 0 must give beta*C without reading A, B"
    C = C0.copy(order="F")
    oracle.dgemm("N", "N", 0.0, An, Bn, 0.0, C, lib=lib)
    assert np.array_equal(C, np.zeros((m, n))), "alpha = beta = 0 gives zeros"
    C = np.full((m, n), np.nan, order="F")
    oracle.dgemm("N", "N", 0.0, An, Bn, 1.0, C, lib=lib)
    assert np.isnan(C).all(), "quick return must leave C untouched"
    C = C0.copy(order="F")
    oracle.dgemm_raw("N", "N", m, n, 0, 1.0, An.ravel(order="F"), m, Bn.ravel(order="F"), 1,
                     -0.5, cf := C.ravel(order="F"), m, lib=lib)
    assert np.array_equal(cf.reshape((m, n), order="F"), -0.5 * C0), "k = 0 gives beta*C"


def pin_dgemm_batched_matches_single(lib, seed=17):
    """The OpenMP batched entry equals a loop of single calls bit for bit,
    with strides larger than the matrices (gaps hold NaN)."""
    g = _rng(seed)
    m, n, k, batch = 6, 5, 7, 9
    lda, ldb, ldc = m + 1, k + 2, m + 3
    sA, sB, sC = lda * k + 5, ldb * k + 1, ldc * n + 4  # B is stored n x k (op(B) = B^T)
    A = g.uniform(-1, 1, size=sA * batch)
    B = g.uniform(-1, 1, size=sB * batch)
    C = g.uniform(-1, 1, size=sC * batch)
    C1 = C.copy()
    oracle.dgemm_strided_batched("N", "T", m, n, k, 1.5, A, lda, sA, B, ldb, sB, -1.0, C1, ldc, sC,
                                 batch, nthreads=4, lib=lib)
    # op(B) = B^T needs B stored n x k: use ldb >= n (here k+2 >= n)
    C2 = C.copy()
    for b in range(batch):
        cv = C2[b * sC:(b + 1) * sC]
        oracle.dgemm_raw("N", "T", m, n, k, 1.5, A[b * sA:(b + 1) * sA], lda,
                         B[b * sB:(b + 1) * sB], ldb, -1.0, cv, ldc, lib=lib)
    assert np.array_equal(C1, C2)


# ----------------------------------------------------------------------------
# dpotrf 'L'
# ----------------------------------------------------------------------------

def _spd(g, n):
    M = g.uniform(-1, 1, size=(n, n))
    S = M @ M.T
    S = 0.5 * (S + S.T) + n * np.eye(n)
    return np.asfortranarray(S)


def pin_potrf_info_closed_form(lib, seed=21):
    """SPD A with a_jj := -1: columns p < j never read a_jj and the pivot of
    column j is -1 - sum l_jp^2 <= -1, so info = j+1 for any correct algorithm."""
    g = _rng(seed)
    for n in (1, 2, 5, 16, 33):
        for j in sorted({0, n - 1, int(g.integers(0, n))}):
            A = _spd(g, n)
            A[j, j] = -1.0
            info = oracle.dpotrf_l(A, lib=lib)
            assert info == j + 1, f"n={n} j={j}: info {info}"


def pin_potrf_nan_zero_tiny(lib):
    """NaN and zero pivots fail (info = j+1); a tiny positive pivot passes."""
    for bad, expect_fail in ((np.nan, True), (0.0, True), (-0.0, True), (1e-300, False)):
        A = np.asfortranarray(np.eye(4))
        A[2, 2] = bad
        info = oracle.dpotrf_l(A, lib=lib)
        assert (info == 3) if expect_fail else (info == 0), f"pivot {bad}: info {info}"
    A = np.asfortranarray(np.eye(3))
    A[1, 1] = np.nan
    A[2, 1] = 5.0
    assert oracle.dpotrf_l(A, lib=lib) == 2


def pin_potrf_exact_integer_factor(lib, seed=22):
    """A = L0 L0^T, L0 integer lower with diagonal in {1, 2, 4} and
    off-diagonal in [-3, 3]: every intermediate is an integer, square roots
    are of perfect squares and divisions are by powers of two, so the factor
    is L0 exactly."""
    g = _rng(seed)
    for n in (1, 3, 8, 17, 40, 64):
        L0 = np.tril(g.integers(-3, 4, size=(n, n)), -1) + np.diag(g.choice([1, 2, 4], size=n))
        A = np.asfortranarray((L0 @ L0.T).astype(np.float64))
        assert np.abs(L0 @ L0.T).max() < 2 ** 50
        info = oracle.dpotrf_l(A, lib=lib)
        assert info == 0
        assert np.array_equal(np.tril(A), L0.astype(np.float64)), f"n={n}"


def pin_potrf_identity_and_diagonal(lib):
    A = np.asfortranarray(np.eye(6))
    assert oracle.dpotrf_l(A, lib=lib) == 0 and np.array_equal(A, np.eye(6))
    d = np.array([1.0, 4.0, 9.0, 0.25, 16.0, 2.25])
    A = np.asfortranarray(np.diag(d))
    assert oracle.dpotrf_l(A, lib=lib) == 0
    assert np.array_equal(A, np.diag(np.sqrt(d)))


def pin_potrf_golden(lib):
    """Textbook 3x3 and Pascal n=8 fixtures, plus Pascal up to n=25 from the
    binomial closed form (all intermediates are integers below 2^53)."""
    for name in ("chol3_textbook.txt", "pascal8_chol.txt"):
        A, L = _load_pair(name)
        X = np.asfortranarray(A.copy())
        assert oracle.dpotrf_l(X, lib=lib) == 0
        assert np.array_equal(np.tril(X), L), name
    for n in (12, 25):
        P = np.array([[math.comb(i + j, i) for j in range(n)] for i in range(n)], dtype=np.float64)
        L = np.array([[math.comb(i, j) for j in range(n)] for i in range(n)], dtype=np.float64)
        X = np.asfortranarray(P)
        assert oracle.dpotrf_l(X, lib=lib) == 0
        assert np.array_equal(np.tril(X), L), f"pascal {n}"


def pin_potrf_small_closed_forms(lib, seed=23):
    """n = 1: l = sqrt(a).  n = 2: l11 = sqrt(a11), l21 = a21/l11,
    l22 = sqrt(a22 - l21^2); the oracle evaluates exactly these operations."""
    g = _rng(seed)
    for _ in range(20):
        a = float(g.uniform(0.1, 10))
        X = np.asfortranarray([[a]])
        assert oracle.dpotrf_l(X, lib=lib) == 0 and X[0, 0] == math.sqrt(a)
        A = _spd(g, 2)
        X = A.copy(order="F")
        assert oracle.dpotrf_l(X, lib=lib) == 0
        l11 = math.sqrt(A[0, 0])
        l21 = A[1, 0] / l11
        l22 = math.sqrt(A[1, 1] - l21 * l21)
        assert X[0, 0] == l11 and X[1, 0] == l21 and X[1, 1] == l22


def pin_potrf_lapack_and_residual(lib, seed=24):
    """Against LAPACK dpotrf (SciPy) and the reconstruction residual, computed
    in extended precision, on the sweep's SPD recipe."""
    from scipy.linalg import lapack
    g = _rng(seed)
    for n in (8, 16, 31, 64, 100):
        A = _spd(g, n)
        X = A.copy(order="F")
        info = oracle.dpotrf_l(X, lib=lib)
        ref, rinfo = lapack.dpotrf(A.copy(order="F"), lower=1, clean=1)
        assert info == rinfo == 0
        L = np.tril(X)
        err = np.linalg.norm(L - ref) / np.linalg.norm(ref)
        assert err <= 1e-13, f"n={n} lapack diff {err}"
        Ll = L.astype(np.longdouble)
        res = np.sqrt(((A.astype(np.longdouble) - Ll @ Ll.T) ** 2).sum()) / np.sqrt(
            (A.astype(np.longdouble) ** 2).sum())
        assert float(res) <= 1e-14, f"n={n} residual {float(res)}"
        # LAPACK's info convention on a failing instance
        A[n // 2, n // 2] = -1.0
        _, rinfo = lapack.dpotrf(A.copy(order="F"), lower=1)
        assert oracle.dpotrf_l(A.copy(order="F"), lib=lib) == rinfo == n // 2 + 1


def pin_potrf_upper_untouched(lib, seed=25):
    """The strict upper triangle (NaN sentinels) and ld padding stay bit-identical."""
    g = _rng(seed)
    n, ld = 12, 15
    A = np.full((ld, n), np.nan, order="F")
    A[:n, :n] = _spd(g, n)
    A[:n, :n][np.triu_indices(n, 1)] = np.nan
    flat = A.ravel(order="F").copy()
    info = oracle.dpotrf_l_raw(n, flat, ld, lib=lib)
    X = flat.reshape(A.shape, order="F")
    assert info == 0
    up = np.triu_indices(n, 1)
    assert np.isnan(X[:n, :n][up]).all() and np.isnan(X[n:]).all()
    assert np.isfinite(np.tril(X[:n, :n])).all()


def pin_potrf_batched_matches_single(lib, seed=26):
    g = _rng(seed)
    n, batch, ld = 9, 11, 10
    s = ld * n + 3
    A = np.full(s * batch, np.nan)
    for b in range(batch):
        blk = np.full((ld, n), np.nan, order="F")
        blk[:n] = _spd(g, n)
        A[b * s:b * s + ld * n] = blk.ravel(order="F")
    A[5 * s + 3 * ld + 3] = -1.0  # instance 5, a_33 = -1 -> info 4
    A1 = A.copy()
    info = oracle.dpotrf_l_strided_batched(n, A1, ld, s, batch, nthreads=4, lib=lib)
    A2 = A.copy()
    info2 = [oracle.dpotrf_l_raw(n, A2[b * s:(b + 1) * s], ld, lib=lib) for b in range(batch)]
    assert list(info) == info2 and info[5] == 4 and sum(info) == 4
    assert np.array_equal(A1, A2, equal_nan=True)


# ----------------------------------------------------------------------------
# Cholesky adjoint
# ----------------------------------------------------------------------------

def _chol(A, lib):
    X = np.asfortranarray(A.copy())
    info = oracle.dpotrf_l(X, lib=lib)
    assert info == 0
    return np.tril(X)


def pin_adjoint_logdet(lib, seed=31):
    """f = log det A = 2 sum log l_ii has Lbar = diag(2 / l_ii), for which
    Phi(L^T Lbar) = I and the gradient is A^{-1} (numpy.linalg.inv)."""
    g = _rng(seed)
    for n in (1, 4, 16, 37):
        A = _spd(g, n)
        L = _chol(A, lib)
        Lbar = np.diag(2.0 / np.diag(L))
        Ab = oracle.dpotrf_l_adjoint(L, Lbar, lib=lib)
        ref = np.linalg.inv(A)
        err = np.linalg.norm(Ab - ref) / np.linalg.norm(ref)
        assert err <= 1e-12, f"n={n}: {err}"


def pin_adjoint_n1(lib):
    for a, lb in ((4.0, 3.0), (2.0, -1.0), (0.25, 0.5)):
        L = np.array([[math.sqrt(a)]])
        Ab = oracle.dpotrf_l_adjoint(L, np.array([[lb]]), lib=lib)
        assert abs(Ab[0, 0] - lb / (2.0 * math.sqrt(a))) <= 1e-15 * abs(Ab[0, 0])


def pin_adjoint_finite_differences(lib, seed=32, h=1e-6):
    """Central differences of f(A) = <W, chol(A)> along symmetric directions."""
    g = _rng(seed)
    for n in (3, 10, 24):
        A = _spd(g, n)
        W = np.tril(g.uniform(-1, 1, size=(n, n)))
        L = _chol(A, lib)
        Ab = oracle.dpotrf_l_adjoint(L, W, lib=lib)
        assert np.array_equal(Ab, Ab.T), "Abar must be symmetric"
        for _ in range(5):
            D = g.uniform(-1, 1, size=(n, n))
            D = 0.5 * (D + D.T)
            fp = np.sum(W * _chol(A + h * D, lib))
            fm = np.sum(W * _chol(A - h * D, lib))
            fd = (fp - fm) / (2 * h)
            an = np.sum(Ab * D)
            assert abs(fd - an) <= 1e-6 * (abs(fd) + 1e-300) + 1e-9, f"n={n}: fd {fd} vs {an}"


def pin_adjoint_batched_matches_single(lib, seed=33):
    """The strided-batched adjoint equals a loop of single adjoints bit for bit
    when L, Lbar and Abar each have their own leading dimension and instance
    stride, with NaN in every gap between instances and in every ld padding:
    a stride or ld taken from the wrong operand, or an instance skipped, reads
    a NaN (or writes the wrong place) and fails."""
    g = _rng(seed)
    n, batch = 7, 5
    lds = {"L": n + 2, "Lb": n + 5, "Ab": n + 1}
    strides = {"L": lds["L"] * n + 3, "Lb": lds["Lb"] * n + 11, "Ab": lds["Ab"] * n + 6}
    bufs = {k: np.full(strides[k] * batch, np.nan) for k in lds}
    Ls, Lbs = [], []
    for b in range(batch):
        L = _chol(_spd(g, n), lib)
        W = np.tril(g.uniform(-1, 1, size=(n, n)))
        Ls.append(L)
        Lbs.append(W)
        for key, M in (("L", L), ("Lb", W)):
            blk = np.full((lds[key], n), np.nan, order="F")
            blk[:n] = M
            blk[:n][np.triu_indices(n, 1)] = np.nan  # strict upper parts are never read
            bufs[key][b * strides[key]:b * strides[key] + lds[key] * n] = blk.ravel(order="F")
    Ab = bufs["Ab"].copy()
    oracle.dpotrf_l_adjoint_strided_batched(n, bufs["L"], lds["L"], strides["L"], bufs["Lb"],
                                            lds["Lb"], strides["Lb"], Ab, lds["Ab"],
                                            strides["Ab"], batch, nthreads=3, lib=lib)
    expect = bufs["Ab"].copy()
    for b in range(batch):
        ref = oracle.dpotrf_l_adjoint(Ls[b], Lbs[b], lib=lib)
        blk = expect[b * strides["Ab"]:b * strides["Ab"] + lds["Ab"] * n].reshape(
            (lds["Ab"], n), order="F").copy(order="F")
        blk[:n] = ref
        expect[b * strides["Ab"]:b * strides["Ab"] + lds["Ab"] * n] = blk.ravel(order="F")
    assert np.isfinite(ref).all()
    assert np.array_equal(Ab, expect, equal_nan=True)


# ---------------------------------------------------------------- dtrmm / dsyrk


def pin_trmm_exact_bruteforce(lib, seed=41):
    """B <= alpha * B * tril(A): exact integer results, A's upper part and B's
    padding rows hold NaN sentinels that must be neither read nor written."""
    g = _rng(seed)
    for m in range(0, 5):
        for n in range(0, 5):
            for alpha in (1.0, -2.0, 0.5):
                A = np.full((n + 2, max(n, 1)), np.nan, order="F")
                for j in range(n):
                    for i in range(j, n):
                        A[i, j] = float(g.integers(-4, 5))
                B, ldb = _colmajor_padded(g, m, n, 2)
                B0 = B.copy(order="F")
                lib.oracle_dtrmm_rlnn(m, n, alpha, oracle._ptr(A), n + 2, oracle._ptr(B), ldb)
                for i in range(m):
                    for j in range(n):
                        exact = Fraction(alpha) * sum(Fraction(B0[i, p]) * Fraction(A[p, j])
                                                      for p in range(j, n))
                        assert B[i, j] == float(exact), (m, n, alpha, i, j)
                assert np.all(np.isnan(B[m:, :])), "padding rows of B written"


def pin_syrk_exact_bruteforce(lib, seed=42):
    """Lower triangle of alpha * A A^T + beta * C exactly; the strictly upper
    triangle (NaN) untouched; beta == 0 does not read C."""
    g = _rng(seed)
    for n in range(0, 5):
        for k in range(0, 5):
            for alpha, beta in ((1.0, 1.0), (-1.0, 2.0), (2.0, 0.0), (0.0, 3.0), (1.0, 0.0)):
                A, lda = _colmajor_padded(g, n, k, 1)
                C = np.full((n + 1, max(n, 1)), np.nan, order="F")
                for j in range(n):
                    for i in range(j, n):
                        C[i, j] = np.nan if beta == 0.0 else float(g.integers(-4, 5))
                C0 = C.copy(order="F")
                lib.oracle_dsyrk_ln(n, k, alpha, oracle._ptr(A), lda, beta, oracle._ptr(C), n + 1)
                for j in range(n):
                    for i in range(n):
                        if i < j:
                            assert np.isnan(C[i, j]), "upper triangle written"
                            continue
                        s = sum(Fraction(A[i, p]) * Fraction(A[j, p]) for p in range(k))
                        exact = Fraction(alpha) * s
                        if beta != 0.0:
                            exact += Fraction(beta) * Fraction(C0[i, j])
                        if (alpha == 0.0 or k == 0) and beta == 1.0:
                            exact = Fraction(C0[i, j])
                        assert C[i, j] == float(exact), (n, k, alpha, beta, i, j)


def pin_trmm_syrk_scipy(lib, seed=43):
    """Against SciPy's BLAS dtrmm (side R, lower, no-trans, non-unit) and dsyrk
    (lower, no-trans), an independent library."""
    from scipy.linalg import blas
    g = _rng(seed)
    for m, n in ((7, 5), (1, 9), (33, 17), (12, 1)):
        A = np.asfortranarray(g.uniform(-1, 1, size=(n, n)))
        B = np.asfortranarray(g.uniform(-1, 1, size=(m, n)))
        ref = blas.dtrmm(0.75, A, B, side=1, lower=1, trans_a=0, diag=0)
        got = B.copy(order="F")
        oracle.dtrmm_rlnn(0.75, A, got, lib=lib)
        assert np.max(np.abs(got - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref))) * n
    for n, k in ((6, 4), (1, 7), (31, 9), (9, 1)):
        A = np.asfortranarray(g.uniform(-1, 1, size=(n, k)))
        C = np.asfortranarray(g.uniform(-1, 1, size=(n, n)))
        ref = blas.dsyrk(-0.5, A, beta=1.5, c=C, trans=0, lower=1)
        got = C.copy(order="F")
        oracle.dsyrk_ln(-0.5, A, 1.5, got, lib=lib)
        lo = np.tril_indices(n)
        assert np.max(np.abs(got[lo] - ref[lo])) <= 1e-14 * max(1.0, np.max(np.abs(ref))) * k
        up = np.triu_indices(n, 1)
        assert np.array_equal(got[up], C[up])


# ---------------------------------------------------------------- Riccati


def _riccati_problem(g, nx, nu, N, rho=None):
    """Stage data with [R S; S^T Q] SPD and BAt = [B^T; A^T]; rho scales A."""
    m = nu + nx
    BAt = g.uniform(-1, 1, size=(N, m, nx)) / math.sqrt(max(nx, 1))
    if rho is not None:
        BAt[:, nu:, :] *= rho
    W = g.uniform(-1, 1, size=(N, m, m))
    RSQ = W @ np.swapaxes(W, 1, 2) / m + np.eye(m)
    V = g.uniform(-1, 1, size=(nx, nx))
    QN = V @ V.T / max(nx, 1) + np.eye(nx)
    return BAt, RSQ, QN


def _split(BAt_n, RSQ_n, nu):
    B = BAt_n[:nu, :].T          # nx x nu
    A = BAt_n[nu:, :].T          # nx x nx
    R = RSQ_n[:nu, :nu]
    S = np.tril(RSQ_n)[nu:, :nu].T   # nu x nx (lower triangle is the stored part)
    Q = RSQ_n[nu:, nu:]
    Q = np.tril(Q) + np.tril(Q, -1).T
    return A, B, R, S, Q


def pin_riccati_closed_form(lib, seed=44):
    """Every stage: Lc_n Lc_n^T equals the Riccati update
    Q + A^T P A - (S^T + A^T P B)(R + B^T P B)^{-1}(S + B^T P A) with
    P = Lc_{n+1} Lc_{n+1}^T (a general solve, not a Cholesky), and the other
    blocks of the stage factor satisfy Lambda Lambda^T = R + B^T P B,
    L_n Lambda^T = S^T + A^T P B.  Also Lc_N Lc_N^T = Q_N."""
    g = _rng(seed)
    for nx, nu, N in ((1, 1, 3), (3, 2, 4), (8, 4, 10), (5, 0, 3), (17, 9, 5), (24, 12, 3)):
        BAt, RSQ, QN = _riccati_problem(g, nx, nu, N)
        F, LN, info = oracle.riccati(BAt, RSQ, QN, nu, lib=lib)
        assert np.all(info == 0)
        assert np.allclose(np.triu(LN, 1), 0.0) and np.allclose(np.triu(F, 1), 0.0)
        assert np.max(np.abs(LN @ LN.T - QN)) <= 1e-13 * np.max(np.abs(QN))
        Lc = LN
        for n in range(N - 1, -1, -1):
            A, B, R, S, Q = _split(BAt[n], RSQ[n], nu)
            P = Lc @ Lc.T
            Fn = F[n]
            Lam, Ln, Lcn = Fn[:nu, :nu], Fn[nu:, :nu], Fn[nu:, nu:]
            if nu > 0:
                Re = R + B.T @ P @ B
                Ge = S.T + A.T @ P @ B
                Pn = Q + A.T @ P @ A - Ge @ np.linalg.solve(Re, Ge.T)
                assert np.max(np.abs(Lam @ Lam.T - Re)) <= 1e-12 * np.max(np.abs(Re))
                assert np.max(np.abs(Ln @ Lam.T - Ge)) <= 1e-12 * np.max(np.abs(Ge))
            else:
                Pn = Q + A.T @ P @ A
            err = np.max(np.abs(Lcn @ Lcn.T - Pn)) / np.max(np.abs(Pn))
            assert err <= 1e-12, (nx, nu, n, err)
            Lc = Lcn


def pin_riccati_scalar(lib):
    """nx = nu = 1: p_n = q + a^2 p - (s + a p b)^2 / (r + b^2 p), Lc_n = sqrt(p_n)."""
    a, b, q, r, s, qN, N = 0.9, 0.7, 1.3, 0.8, 0.2, 2.0, 6
    BAt = np.array([[[b], [a]]] * N)
    RSQ = np.array([[[r, s], [s, q]]] * N)
    F, LN, info = oracle.riccati(BAt, RSQ, np.array([[qN]]), 1, lib=lib)
    assert np.all(info == 0)
    p = qN
    assert abs(LN[0, 0] - math.sqrt(p)) <= 1e-15 * math.sqrt(p)
    for n in range(N - 1, -1, -1):
        lam = math.sqrt(r + b * b * p)
        l = (s + a * p * b) / lam
        p = q + a * a * p - (s + a * p * b) ** 2 / (r + b * b * p)
        assert abs(F[n][0, 0] - lam) <= 4e-16 * lam
        assert abs(F[n][1, 0] - l) <= 8e-16 * abs(l)
        assert abs(F[n][1, 1] - math.sqrt(p)) <= 8e-16 * math.sqrt(p), n


def pin_riccati_dare_limit(lib, seed=45):
    """Time-invariant stages over a long horizon: P_0 converges to the
    stabilizing solution of the discrete algebraic Riccati equation
    (SciPy's solve_discrete_are, s = the cross term S^T)."""
    from scipy.linalg import solve_discrete_are
    g = _rng(seed)
    for nx, nu in ((4, 2), (6, 3)):
        BAt1, RSQ1, _ = _riccati_problem(g, nx, nu, 1, rho=0.6)
        N = 120
        BAt = np.repeat(BAt1, N, axis=0)
        RSQ = np.repeat(RSQ1, N, axis=0)
        A, B, R, S, Q = _split(BAt1[0], RSQ1[0], nu)
        F, LN, info = oracle.riccati(BAt, RSQ, np.eye(nx), nu, lib=lib)
        assert np.all(info == 0)
        Lc = F[0][nu:, nu:]
        X = solve_discrete_are(A, B, Q, R, s=S.T)
        assert np.max(np.abs(Lc @ Lc.T - X)) <= 1e-10 * np.max(np.abs(X)), (nx, nu)


def pin_riccati_info(lib, seed=46):
    """A stage whose matrix is not positive definite at column j reports
    info = j + 1 there; the stages after it in the recursion (lower n) are not
    computed (info -1, F untouched); a bad Q_N stops everything."""
    g = _rng(seed)
    nx, nu, N = 5, 3, 6
    m = nx + nu
    for fail_stage, j in ((3, 0), (0, 6), (5, 2)):
        BAt, RSQ, QN = _riccati_problem(g, nx, nu, N)
        RSQ[fail_stage] = np.diag(np.arange(1.0, m + 1))
        RSQ[fail_stage][j, j] = -1.0
        BAt[fail_stage][j, :] = 0.0
        bat = np.ascontiguousarray(np.swapaxes(BAt, 1, 2))
        rsq = np.ascontiguousarray(np.swapaxes(RSQ, 1, 2))
        q = np.asfortranarray(QN)
        F = np.full((N, m, m), 7.0)
        LN = np.zeros((nx, nx), order="F")
        info = np.zeros(N + 1, dtype=np.int32)
        lib.oracle_riccati(nx, nu, N, oracle._ptr(bat), m, m * nx, oracle._ptr(rsq), m, m * m,
                           oracle._ptr(q), nx, oracle._ptr(F), m, m * m, oracle._ptr(LN), nx,
                           oracle._ptr(info))
        want = [-1] * fail_stage + [j + 1] + [0] * (N - fail_stage)
        assert info.tolist() == want, (info.tolist(), want)
        for n in range(fail_stage):
            assert np.all(F[n] == 7.0), "stage after a failure was written"
    BAt, RSQ, QN = _riccati_problem(g, nx, nu, N)
    QN[2, 2] = -5.0
    F, LN, info = oracle.riccati(BAt, RSQ, QN, nu, lib=lib)
    assert info.tolist() == [-1] * N + [3]


def pin_riccati_batched_matches_single(lib, seed=47):
    """The batched wrapper with padded leading dimensions and problem strides
    reproduces the single-problem results bit for bit."""
    g = _rng(seed)
    nx, nu, N, batch = 6, 3, 4, 3
    m = nx + nu
    ldb, ldr, ldq, ldf, ldl = m + 1, m + 2, nx + 3, m + 1, nx + 2
    sb, sr, sf = ldb * nx + 5, ldr * m + 1, ldf * m + 3
    BATS = np.zeros(batch * N * sb + 64)
    RSQS = np.zeros(batch * N * sr + 64)
    QS = np.zeros(batch * ldq * nx + 64)
    probs = []
    for b in range(batch):
        BAt, RSQ, QN = _riccati_problem(g, nx, nu, N)
        probs.append((BAt, RSQ, QN))
        for n in range(N):
            for j in range(nx):
                o = b * N * sb + n * sb + j * ldb
                BATS[o:o + m] = BAt[n][:, j]
            for j in range(m):
                o = b * N * sr + n * sr + j * ldr
                RSQS[o:o + m] = RSQ[n][:, j]
        for j in range(nx):
            o = b * ldq * nx + j * ldq
            QS[o:o + nx] = QN[:, j]
    FS = np.zeros(batch * N * sf + 64)
    LS = np.zeros(batch * ldl * nx + 64)
    info = np.zeros(batch * (N + 1), dtype=np.int32)
    oracle.riccati_strided_batched(nx, nu, N, BATS, ldb, sb, N * sb, RSQS, ldr, sr, N * sr, QS,
                                   ldq, ldq * nx, FS, ldf, sf, N * sf, LS, ldl, ldl * nx, info,
                                   batch, lib=lib)
    assert np.all(info == 0)
    for b, (BAt, RSQ, QN) in enumerate(probs):
        F, LN, _ = oracle.riccati(BAt, RSQ, QN, nu, lib=lib)
        for n in range(N):
            for j in range(m):
                o = b * N * sf + n * sf + j * ldf
                assert np.array_equal(FS[o + j:o + m], F[n][j:, j])
        for j in range(nx):
            o = b * ldl * nx + j * ldl
            assert np.array_equal(LS[o + j:o + nx], LN[j:, j])


ALL_PINS = [
    pin_dgemm_exact_bruteforce,
    pin_dgemm_lowercase_and_conj_flags,
    pin_dgemm_closed_forms,
    pin_dgemm_transposition_rule,
    pin_dgemm_scipy,
    pin_dgemm_special_scalars,
    pin_dgemm_batched_matches_single,
    pin_potrf_info_closed_form,
    pin_potrf_nan_zero_tiny,
    pin_potrf_exact_integer_factor,
    pin_potrf_identity_and_diagonal,
    pin_potrf_golden,
    pin_potrf_small_closed_forms,
    pin_potrf_lapack_and_residual,
    pin_potrf_upper_untouched,
    pin_potrf_batched_matches_single,
    pin_adjoint_logdet,
    pin_adjoint_n1,
    pin_adjoint_finite_differences,
    pin_adjoint_batched_matches_single,
    pin_trmm_exact_bruteforce,
    pin_syrk_exact_bruteforce,
    pin_trmm_syrk_scipy,
    pin_riccati_closed_form,
    pin_riccati_scalar,
    pin_riccati_dare_limit,
    pin_riccati_info,
    pin_riccati_batched_matches_single,
]
