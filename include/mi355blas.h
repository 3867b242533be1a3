/*
 * mi355blas.h -- C ABI of an MI355X (gfx950) library for small FP64 matrices:
 * column-major BLAS dgemm and LAPACK lower dpotrf, plain, strided-batched and
 * pointer-array-batched.
 *
 * The operations are those of Frison, Sartor, Zanelli, Diehl, "The BLAS API of
 * BLASFEO: optimizing performance for small matrices" (arXiv:1902.08115):
 *   - dgemm: Sec. 2.1 defines C <= A*B + C on column-major operands and elides
 *     the transposition options, the scalars alpha/beta and the leading
 *     dimensions for readability; this library restores the standard BLAS
 *     form  C <= alpha*op(A)*op(B) + beta*C  (the form written out for
 *     variant 'D' in Sec. 2.2; the four trans cases of App. D, Table 3).
 *   - dpotrf 'L': Sec. 3.1.5 (lower Cholesky factor A = L*L^T, L overwriting
 *     the lower triangle).
 * The size switch between a direct (no staging) kernel for tiny operands and
 * an LDS-staged, packed kernel above a measured crossover follows the
 * variant-switching scheme of Sec. 2.4 and Sec. 3.1.
 *
 * Conventions common to every call
 *   - Integers m, n, k, ld*, batch are 32-bit int; strides are int64_t and
 *     count elements.  Matrix X with leading dimension ldx holds element (i,j)
 *     at X[i + j*ldx].
 *   - trans characters: 'N','n' (no transpose), 'T','t','C','c' (transpose;
 *     'C' == 'T' for real data).  uplo: 'L','l'.  'U','u' is recognised but not
 *     implemented (MB_ERR_UNSUPPORTED).
 *   - Return value: MB_OK (0), or -i when argument i (1-based position in that
 *     function's own argument list) is illegal, or MB_ERR_UNSUPPORTED, or
 *     MB_ERR_HIP when a HIP launch fails.  Arguments are validated on the host
 *     before anything is launched; an illegal call launches nothing, writes
 *     nothing and prints nothing.
 *   - Memory: every matrix, pointer array and info array is caller-owned
 *     DEVICE memory.  No call allocates device or host memory, and no call
 *     synchronizes: work is enqueued on `stream` (0 = null stream) and results
 *     are valid once that stream has completed it.
 *   - Numerical failure of dpotrf is reported only through the device array
 *     info[] (LAPACK convention), readable after the stream completes.
 *   - Calls are reentrant: the library keeps no mutable global state.
 *   - Aliasing: C must not overlap A or B, and distinct batch instances of C
 *     (or of A in dpotrf) must not overlap; otherwise results are undefined.
 *     Input strides (strideA, strideB of dgemm) may be 0 (broadcast).
 */
#ifndef MI355BLAS_H
#define MI355BLAS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MB_OK 0
#define MB_ERR_HIP (-1000)
#define MB_ERR_UNSUPPORTED (-1001)

/* Kernel family selection for the *_ex calls. */
#define MB_VARIANT_AUTO 0   /* measured size switch (what the plain calls use) */
#define MB_VARIANT_DIRECT 1 /* operands read straight into registers, no LDS   */
#define MB_VARIANT_PACKED 2 /* operand panels staged (and transposed) in LDS,  */
                            /* FP64 MFMA rank-4 updates                        */

/* ---------------------------------------------------------------- dgemm --- */

/*
 * C <= alpha*op(A)*op(B) + beta*C  (Sec. 2.1 with the BLAS scalars; Sec. 2.2).
 *   transa, transb  op(X) = X ('N') or X^T ('T'/'C').           positions 1, 2
 *   m, n            rows and columns of C (>= 0).                positions 3, 4
 *   k               inner dimension (>= 0).                      position 5
 *   alpha           scalar (by value).                           position 6
 *   A               op(A) is m x k; A is m x k ('N') or k x m ('T'), lda >=
 *                   max(1, rows of A).                           positions 7, 8
 *   B               op(B) is k x n; B is k x n ('N') or n x k ('T'), ldb >=
 *                   max(1, rows of B).                           positions 9, 10
 *   beta            scalar.                                      position 11
 *   C               m x n, in/out, ldc >= max(1, m).             positions 12, 13
 *   stream          HIP stream.                                  position 14
 * beta == 0: C is not read (NaN/Inf in C do not propagate).  alpha == 0 or
 * k == 0: A and B are not read and C <= beta*C.  Quick return (nothing
 * launched, C untouched): m == 0, n == 0, or (alpha == 0 or k == 0) and
 * beta == 1.  Rows m..ldc-1 of C are never touched.
 */
int mb_dgemm(char transa, char transb, int m, int n, int k, double alpha,
             const double *A, int lda, const double *B, int ldb, double beta,
             double *C, int ldc, hipStream_t stream);

/*
 * Strided batch: instance b uses A + b*strideA, B + b*strideB, C + b*strideC.
 * Argument positions: transa 1, transb 2, m 3, n 4, k 5, alpha 6, A 7, lda 8,
 * strideA 9, B 10, ldb 11, strideB 12, beta 13, C 14, ldc 15, strideC 16,
 * batch 17, stream 18.  Strides must be >= 0; strideC must keep instances of C
 * disjoint (strideC >= ldc*(n-1)+m when batch > 1).  batch == 0 is a quick
 * return.  Every instance is computed exactly as the single call would compute
 * it (the kernel choice depends on (trans, m, n, k) only).
 */
int mb_dgemm_strided_batched(char transa, char transb, int m, int n, int k, double alpha,
                             const double *A, int lda, int64_t strideA,
                             const double *B, int ldb, int64_t strideB, double beta,
                             double *C, int ldc, int64_t strideC, int batch,
                             hipStream_t stream);

/*
 * Pointer-array batch: instance b uses Aarray[b], Barray[b], Carray[b]; the
 * three arrays of batch pointers are themselves in device memory.
 * Positions: transa 1, transb 2, m 3, n 4, k 5, alpha 6, Aarray 7, lda 8,
 * Barray 9, ldb 10, beta 11, Carray 12, ldc 13, batch 14, stream 15.
 */
int mb_dgemm_batched(char transa, char transb, int m, int n, int k, double alpha,
                     const double *const *Aarray, int lda, const double *const *Barray, int ldb,
                     double beta, double *const *Carray, int ldc, int batch, hipStream_t stream);

/* As the strided / pointer-array calls, with an explicit kernel family
 * (MB_VARIANT_*) inserted before `stream` (its position is then the
 * second-to-last).  Used to measure both sides of the size switch. */
int mb_dgemm_strided_batched_ex(char transa, char transb, int m, int n, int k, double alpha,
                                const double *A, int lda, int64_t strideA,
                                const double *B, int ldb, int64_t strideB, double beta,
                                double *C, int ldc, int64_t strideC, int batch, int variant,
                                hipStream_t stream);
int mb_dgemm_batched_ex(char transa, char transb, int m, int n, int k, double alpha,
                        const double *const *Aarray, int lda, const double *const *Barray,
                        int ldb, double beta, double *const *Carray, int ldc, int batch,
                        int variant, hipStream_t stream);

/* Tuning entry: the strided batch on one forced configuration of the packed
 * kernel menu, 0 <= config < mb_dgemm_config_count() (position 18; returns
 * MB_ERR_UNSUPPORTED when a one-wave-per-instance configuration cannot hold
 * the m x n result).  The autotuner measures the menu with it. */
int mb_dgemm_strided_batched_config(char transa, char transb, int m, int n, int k,
                                    double alpha, const double *A, int lda, int64_t strideA,
                                    const double *B, int ldb, int64_t strideB, double beta,
                                    double *C, int ldc, int64_t strideC, int batch, int config,
                                    hipStream_t stream);
int mb_dgemm_config_count(void);
/* Static name of a packed configuration ("illegal" when out of range). */
const char *mb_dgemm_config_name(int config);
/* Largest m and n a packed configuration accepts (INT_MAX for the workgroup
 * tile shapes; a one-wave-per-instance shape holds the whole result), -1 for
 * an out-of-range configuration. */
int mb_dgemm_config_max_mn(int config);

/* Host-only query: the kernel family (MB_VARIANT_DIRECT or MB_VARIANT_PACKED)
 * that the plain calls select for this shape, or -1 for an illegal trans. */
int mb_dgemm_select(char transa, char transb, int m, int n, int k);

/* Host-only query: a static name of the kernel class the call would run
 * ("gemm_direct", "gemm_packed_tile64_k16", ...), for attributing profiles; the
 * scalar alpha/beta quick returns are not considered. */
const char *mb_dgemm_kernel_name(char transa, char transb, int m, int n, int k, int variant);

/* --------------------------------------------------------------- dpotrf --- */

/*
 * Lower Cholesky factorization A = L*L^T (Sec. 3.1.5), L overwriting the lower
 * triangle of A; the strict upper triangle is neither read nor written.
 *   uplo   'L' (position 1); 'U' returns MB_ERR_UNSUPPORTED.
 *   n      order (>= 0)                      position 2
 *   A      n x n, in/out, lda >= max(1, n)   positions 3, 4
 *   info   one int in device memory          position 5
 *   stream                                   position 6
 * info (LAPACK convention): 0 on success; j > 0 when the leading minor of
 * order j is not positive definite (the pivot of column j-1 is <= 0 or NaN)
 * and the factorization stopped.  Columns 0..j-2 then hold the valid factor;
 * the rest of the lower triangle is unspecified.  n == 0 sets info to 0.
 */
int mb_dpotrf(char uplo, int n, double *A, int lda, int *info, hipStream_t stream);

/* Strided batch; info[batch] in device memory.  Positions: uplo 1, n 2, A 3,
 * lda 4, strideA 5, info 6, batch 7, stream 8.  strideA >= lda*(n-1)+n when
 * batch > 1. */
int mb_dpotrf_strided_batched(char uplo, int n, double *A, int lda, int64_t strideA, int *info,
                              int batch, hipStream_t stream);

/* Pointer-array batch.  Positions: uplo 1, n 2, Aarray 3, lda 4, info 5,
 * batch 6, stream 7. */
int mb_dpotrf_batched(char uplo, int n, double *const *Aarray, int lda, int *info, int batch,
                      hipStream_t stream);

/* Host-only query: static name of the kernel class used for order n. */
const char *mb_dpotrf_kernel_name(int n);

/* ---------------------------------------------------------------- misc --- */

/* Static text for a status code (never NULL). */
const char *mb_status_string(int status);

/* Library version as major*10000 + minor*100 + patch. */
int mb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MI355BLAS_H */
