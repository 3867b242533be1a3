/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the batched
 * small-matrix FP64 dgemm / dpotrf('L') path and the Riccati recursion built
 * from dtrmm, dsyrk and dpotrf.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP implementation.
 *
 * Precision: IEEE binary64 throughout, compiled without fast-math and with
 * floating-point contraction disabled, so every product and sum below is
 * rounded exactly as written, in the order written.
 *
 * Storage: BLAS column-major (Frison et al., "The BLAS API of BLASFEO",
 * Sec. 2.1 Notation: all of A, B, C are column-major), element (i,j) of a
 * matrix X with leading dimension ldx lives at X[i + j*ldx].
 *
 * Functions and the passage each one follows:
 *   oracle_dgemm                -- Sec. 2.1 (C <= A*B + C) with the standard
 *                                  BLAS scalars and transposition options that
 *                                  the paper elides for readability (Sec. 2.1,
 *                                  and the alpha/beta form used for variant 'D'
 *                                  in Sec. 2.2).  The four trans cases are the
 *                                  ones of Table 3 (App. D).  Plain definition.
 *   oracle_dpotrf_l             -- Sec. 3.1.5 (dpotrf 'L', lower Cholesky
 *                                  factor, the exponent 1/2 of Sec. 5.2).
 *                                  Textbook left-looking column algorithm.
 *   oracle_dpotrf_l_adjoint     -- not in the paper; reverse-mode derivative
 *                                  of the lower Cholesky factor (S. P. Smith,
 *                                  1995; I. Murray, arXiv:1602.07527, 2016).
 *   oracle_dtrmm_rlnn           -- Sec. 3.1.4 and Sec. 5.2 (BLAS dtrmm
 *                                  with side 'R', uplo 'L', trans 'N', diag
 *                                  'N': B <= alpha * B * A, A lower).  Plain
 *                                  definition.
 *   oracle_dsyrk_ln             -- Sec. 3.1.2 and Sec. 5.2 (BLAS dsyrk with
 *                                  uplo 'L', trans 'N': lower triangle of
 *                                  C <= alpha * A * A^T + beta * C).  Plain
 *                                  definition.
 *   oracle_riccati              -- Sec. 5.2, the factorized backward Riccati
 *                                  recursion: per stage one dtrmm_rlnn, one
 *                                  dsyrk_ln and one dpotrf_l, in that order.
 *   *_strided_batched           -- independent instances, OpenMP over
 *                                  instances, each instance single-threaded
 *                                  (the paper evaluates single-threaded
 *                                  libraries, Sec. 4).
 *
 * Parity pins for every function live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int is_notrans(char t) { return t == 'N' || t == 'n'; }

/* op(X)(r, c) for a matrix stored column-major with leading dimension ld:
 * 'N' -> X[r + c*ld], 'T'/'C' -> X[c + r*ld]  (real data: 'C' == 'T'). */
static double op_elem(char t, const double *X, int ld, int r, int c)
{
    if (is_notrans(t))
        return X[(size_t)r + (size_t)c * (size_t)ld];
    return X[(size_t)c + (size_t)r * (size_t)ld];
}

/*
 * C <= alpha * op(A) * op(B) + beta * C   (m x n result, inner length k)
 *
 *   s_ij = sum_{p=0}^{k-1} op(A)(i,p) * op(B)(p,j), summed in increasing p;
 *   beta != 0 : c_ij <= alpha * s_ij + beta * c_ij
 *   beta == 0 : c_ij <= alpha * s_ij            (C is not read)
 *   alpha == 0 or k == 0 : c_ij <= beta * c_ij   (A and B are not read;
 *                                                 zero when beta == 0)
 * Quick return (C untouched): m == 0, n == 0, or (alpha == 0 or k == 0) with
 * beta == 1.  Rows m..ldc-1 of C are never touched.
 * Argument validation is not part of the arithmetic and is not done here.
 */
void oracle_dgemm(char transa, char transb, int m, int n, int k, double alpha,
                  const double *A, int lda, const double *B, int ldb,
                  double beta, double *C, int ldc)
{
    if (m == 0 || n == 0)
        return;
    if ((alpha == 0.0 || k == 0) && beta == 1.0)
        return;
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < m; ++i) {
            double *cij = &C[(size_t)i + (size_t)j * (size_t)ldc];
            if (alpha == 0.0 || k == 0) {
                *cij = (beta == 0.0) ? 0.0 : beta * (*cij);
                continue;
            }
            double s = 0.0;
            for (int p = 0; p < k; ++p)
                s += op_elem(transa, A, lda, i, p) * op_elem(transb, B, ldb, p, j);
            if (beta == 0.0)
                *cij = alpha * s;
            else
                *cij = alpha * s + beta * (*cij);
        }
    }
}

/* Instance b uses A + b*strideA, B + b*strideB, C + b*strideC. */
void oracle_dgemm_strided_batched(char transa, char transb, int m, int n, int k,
                                  double alpha, const double *A, int lda, int64_t strideA,
                                  const double *B, int ldb, int64_t strideB,
                                  double beta, double *C, int ldc, int64_t strideC,
                                  int batch, int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic) num_threads(nthreads)
#endif
    for (int b = 0; b < batch; ++b)
        oracle_dgemm(transa, transb, m, n, k, alpha, A + (ptrdiff_t)b * strideA, lda,
                     B + (ptrdiff_t)b * strideB, ldb, beta, C + (ptrdiff_t)b * strideC, ldc);
    (void)nthreads;
}

/*
 * Lower Cholesky factor, A = L * L^T, L overwriting the lower triangle of A.
 * Column (left-looking) form: for j = 0..n-1
 *   d    = a_jj - sum_{p<j} l_jp^2
 *   if !(d > 0): return j+1          (zero, negative and NaN pivots fail;
 *                                     column j and later are left as they are)
 *   l_jj = sqrt(d)
 *   l_ij = (a_ij - sum_{p<j} l_ip * l_jp) / l_jj      for i = j+1..n-1
 * Returns 0 on success.  Only the lower triangle is read or written.
 */
int oracle_dpotrf_l(int n, double *A, int lda)
{
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j + (size_t)j * (size_t)lda];
        for (int p = 0; p < j; ++p) {
            double ljp = A[(size_t)j + (size_t)p * (size_t)lda];
            d -= ljp * ljp;
        }
        if (!(d > 0.0))
            return j + 1;
        double ljj = sqrt(d);
        A[(size_t)j + (size_t)j * (size_t)lda] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = A[(size_t)i + (size_t)j * (size_t)lda];
            for (int p = 0; p < j; ++p)
                s -= A[(size_t)i + (size_t)p * (size_t)lda] * A[(size_t)j + (size_t)p * (size_t)lda];
            A[(size_t)i + (size_t)j * (size_t)lda] = s / ljj;
        }
    }
    return 0;
}

void oracle_dpotrf_l_strided_batched(int n, double *A, int lda, int64_t strideA,
                                     int *info, int batch, int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic) num_threads(nthreads)
#endif
    for (int b = 0; b < batch; ++b)
        info[b] = oracle_dpotrf_l(n, A + (ptrdiff_t)b * strideA, lda);
    (void)nthreads;
}

/*
 * Reverse-mode derivative of L = chol(A) (lower), for a scalar f(L):
 *   given Lbar = df/dL (only its lower triangle matters, since L is lower),
 *   P    = Phi(L^T * tril(Lbar)),  Phi = lower triangle with the diagonal halved
 *   S    = L^{-T} * P * L^{-1}     (two triangular solves)
 *   Abar = (S + S^T) / 2           (gradient with respect to a symmetric A)
 * Derivation: dA = dL L^T + L dL^T gives L^{-1} dL = Phi(L^{-1} dA L^{-T});
 * Phi is self-adjoint under the Frobenius inner product.
 * L, Lbar are read (lower triangles only); Abar (n x n, full) is written.
 * Returns 0, or -1 when a work buffer cannot be allocated.
 */
int oracle_dpotrf_l_adjoint(int n, const double *L, int ldl, const double *Lbar, int ldlb,
                            double *Abar, int ldab)
{
    if (n == 0)
        return 0;
    double *P = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    if (!P)
        return -1;
#define Lx(i, j) L[(size_t)(i) + (size_t)(j) * (size_t)ldl]
#define LBx(i, j) ((i) >= (j) ? Lbar[(size_t)(i) + (size_t)(j) * (size_t)ldlb] : 0.0)
#define Px(i, j) P[(size_t)(i) + (size_t)(j) * (size_t)n]
    /* P = Phi(L^T * tril(Lbar)) : (L^T Lbar)_ij = sum_p L_pi * Lbar_pj,
     * L_pi nonzero only for p >= i, Lbar_pj only for p >= j.  Only i >= j kept. */
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double v = 0.0;
            if (i >= j) {
                for (int p = i; p < n; ++p)
                    v += Lx(p, i) * LBx(p, j);
                if (i == j)
                    v *= 0.5;
            }
            Px(i, j) = v;
        }
    /* Y = L^{-T} P : solve L^T Y = P column by column (back substitution,
     * L^T is upper triangular with (L^T)_ip = L_pi). Overwrites P with Y. */
    for (int j = 0; j < n; ++j)
        for (int i = n - 1; i >= 0; --i) {
            double v = Px(i, j);
            for (int p = i + 1; p < n; ++p)
                v -= Lx(p, i) * Px(p, j);
            Px(i, j) = v / Lx(i, i);
        }
    /* S = Y L^{-1} : solve S L = Y row by row, i.e. for each row r,
     * sum_{p >= c} S_rp L_pc = Y_rc, back substitution over c = n-1..0.
     * Overwrites P with S. */
    for (int r = 0; r < n; ++r)
        for (int c = n - 1; c >= 0; --c) {
            double v = Px(r, c);
            for (int p = c + 1; p < n; ++p)
                v -= Px(r, p) * Lx(p, c);
            Px(r, c) = v / Lx(c, c);
        }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            Abar[(size_t)i + (size_t)j * (size_t)ldab] = 0.5 * (Px(i, j) + Px(j, i));
#undef Lx
#undef LBx
#undef Px
    free(P);
    return 0;
}

int oracle_dpotrf_l_adjoint_strided_batched(int n, const double *L, int ldl, int64_t strideL,
                                            const double *Lbar, int ldlb, int64_t strideLb,
                                            double *Abar, int ldab, int64_t strideAb,
                                            int batch, int nthreads)
{
    int bad = 0;
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic) num_threads(nthreads) reduction(| : bad)
#endif
    for (int b = 0; b < batch; ++b)
        bad |= oracle_dpotrf_l_adjoint(n, L + (ptrdiff_t)b * strideL, ldl,
                                       Lbar + (ptrdiff_t)b * strideLb, ldlb,
                                       Abar + (ptrdiff_t)b * strideAb, ldab) != 0;
    (void)nthreads;
    return bad ? -1 : 0;
}

/*
 * B <= alpha * B * A, B m x n, A n x n lower triangular with its diagonal
 * (dtrmm side 'R', uplo 'L', trans 'N', diag 'N').  Entry (i, j) of B * A is
 * sum_{p=j}^{n-1} b_ip * a_pj, summed in increasing p (A's strictly upper
 * part is never read).  Columns are produced in increasing j: column j reads
 * only columns p >= j of B, none of which has been overwritten yet.
 */
void oracle_dtrmm_rlnn(int m, int n, double alpha, const double *A, int lda, double *B, int ldb)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int p = j; p < n; ++p)
                s += B[(size_t)i + (size_t)p * (size_t)ldb] * A[(size_t)p + (size_t)j * (size_t)lda];
            B[(size_t)i + (size_t)j * (size_t)ldb] = alpha * s;
        }
}

/*
 * Lower triangle of C <= alpha * A * A^T + beta * C, C n x n, A n x k
 * (dsyrk uplo 'L', trans 'N').  For i >= j, s_ij = sum_{p<k} a_ip * a_jp in
 * increasing p, and c_ij <= alpha * s_ij + beta * c_ij (beta == 0: C not
 * read).  The scalar special cases are those of oracle_dgemm.  The strictly
 * upper triangle of C is never touched.
 */
void oracle_dsyrk_ln(int n, int k, double alpha, const double *A, int lda, double beta,
                     double *C, int ldc)
{
    if (n == 0)
        return;
    if ((alpha == 0.0 || k == 0) && beta == 1.0)
        return;
    for (int j = 0; j < n; ++j)
        for (int i = j; i < n; ++i) {
            double *c = &C[(size_t)i + (size_t)j * (size_t)ldc];
            if (k == 0 || alpha == 0.0) {
                *c = (beta == 0.0) ? 0.0 : beta * (*c);
                continue;
            }
            double acc = 0.0;
            for (int p = 0; p < k; ++p)
                acc += A[(size_t)i + (size_t)p * (size_t)lda] * A[(size_t)j + (size_t)p * (size_t)lda];
            if (beta == 0.0)
                *c = alpha * acc;
            else
                *c = alpha * acc + beta * (*c);
        }
}

/*
 * One backward Riccati recursion in the factorized form of Sec. 5.2, for a
 * system with nx states, nu controls and horizon N (m = nu + nx):
 *   Lc_N = chol(Q_N)                                      (dpotrf_l)
 *   for n = N-1 down to 0:
 *     C_n  = BAt_n * Lc_{n+1}        m x nx               (dtrmm_rlnn)
 *     F_n  = RSQ_n + C_n * C_n^T     lower triangle       (dsyrk_ln)
 *     F_n  = chol(F_n) = [Lambda_n 0; L_n Lc_n]           (dpotrf_l)
 *     Lc_n = F_n(nu:m, nu:m), the lower factor of P_n
 * with BAt_n = [B_n^T; A_n^T] (m x nx) and RSQ_n = [R_n S_n; S_n^T Q_n]
 * (m x m, symmetric, lower triangle read).  Stage n of X is at
 * X + n * sX within the problem.  Outputs: the lower triangles of F_n
 * (ldf) and of LN = Lc_N (ldl); their strictly upper parts are not touched.
 * info[N] is the dpotrf info of Q_N, info[n] that of stage n; a failed
 * factorization stops the recursion, and the stages below it are not
 * computed (F_n untouched, info[n] = -1).
 * Returns 0, or -1 when the work buffer cannot be allocated.
 */
int oracle_riccati(int nx, int nu, int N,
                   const double *BAt, int ldbat, int64_t sbat,
                   const double *RSQ, int ldrsq, int64_t srsq,
                   const double *QN, int ldq,
                   double *F, int ldf, int64_t sf,
                   double *LN, int ldl, int *info)
{
    const int m = nu + nx;
    for (int n = 0; n <= N; ++n)
        info[n] = -1;
    for (int j = 0; j < nx; ++j)
        for (int i = j; i < nx; ++i)
            LN[(size_t)i + (size_t)j * (size_t)ldl] = QN[(size_t)i + (size_t)j * (size_t)ldq];
    info[N] = oracle_dpotrf_l(nx, LN, ldl);
    if (info[N] != 0 || N == 0)
        return 0;
    double *C = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * (size_t)(nx > 0 ? nx : 1));
    if (!C)
        return -1;
    const double *Lc = LN;
    int ldlc = ldl;
    for (int n = N - 1; n >= 0; --n) {
        const double *Bn = BAt + (ptrdiff_t)n * sbat;
        const double *Rn = RSQ + (ptrdiff_t)n * srsq;
        double *Fn = F + (ptrdiff_t)n * sf;
        for (int j = 0; j < nx; ++j)
            for (int i = 0; i < m; ++i)
                C[(size_t)i + (size_t)j * (size_t)m] = Bn[(size_t)i + (size_t)j * (size_t)ldbat];
        oracle_dtrmm_rlnn(m, nx, 1.0, Lc, ldlc, C, m);
        for (int j = 0; j < m; ++j)
            for (int i = j; i < m; ++i)
                Fn[(size_t)i + (size_t)j * (size_t)ldf] = Rn[(size_t)i + (size_t)j * (size_t)ldrsq];
        oracle_dsyrk_ln(m, nx, 1.0, C, m, 1.0, Fn, ldf);
        info[n] = oracle_dpotrf_l(m, Fn, ldf);
        if (info[n] != 0)
            break;
        Lc = Fn + (size_t)nu + (size_t)nu * (size_t)ldf;
        ldlc = ldf;
    }
    free(C);
    return 0;
}

/* Problem b uses X + b * strideX for every operand and info + b * (N + 1). */
int oracle_riccati_strided_batched(int nx, int nu, int N,
                                   const double *BAt, int ldbat, int64_t sbat, int64_t strideBAt,
                                   const double *RSQ, int ldrsq, int64_t srsq, int64_t strideRSQ,
                                   const double *QN, int ldq, int64_t strideQ,
                                   double *F, int ldf, int64_t sf, int64_t strideF,
                                   double *LN, int ldl, int64_t strideL,
                                   int *info, int batch, int nthreads)
{
    int bad = 0;
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic) num_threads(nthreads) reduction(| : bad)
#endif
    for (int b = 0; b < batch; ++b)
        bad |= oracle_riccati(nx, nu, N, BAt + (ptrdiff_t)b * strideBAt, ldbat, sbat,
                              RSQ + (ptrdiff_t)b * strideRSQ, ldrsq, srsq,
                              QN + (ptrdiff_t)b * strideQ, ldq,
                              F + (ptrdiff_t)b * strideF, ldf, sf,
                              LN + (ptrdiff_t)b * strideL, ldl,
                              info + (ptrdiff_t)b * (N + 1)) != 0;
    (void)nthreads;
    return bad ? -1 : 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
