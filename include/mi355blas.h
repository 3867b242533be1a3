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
 *   - the backward Riccati recursion of Sec. 5.2 (dtrmm_rlnn, dsyrk_ln and
 *     dpotrf_l per stage), batched over independent problems.
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
 *     DEVICE memory.  Apart from plan creation and destruction (mb_plan_*),
 *     no call allocates device or host memory, and no call synchronizes: work
 *     is enqueued on `stream` (0 = null stream) and results are valid once
 *     that stream has completed it.
 *   - Numerical failure of dpotrf is reported only through the device array
 *     info[] (LAPACK convention), readable after the stream completes.
 *   - Calls are reentrant: the library keeps no mutable global state (a plan
 *     is state owned by its caller; see mb_plan_create).
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
#define MB_ERR_INVALID_PROBLEM (-1002) /* a plan problem failed validation */
#define MB_ERR_SCRATCH (-1003) /* more device scratch than the allocation-free entry point holds */

/* Kernel family selection for the *_ex calls. */
#define MB_VARIANT_AUTO 0   /* measured size switch (what the plain calls use) */
#define MB_VARIANT_DIRECT 1 /* operands read straight into registers, no LDS   */
#define MB_VARIANT_PACKED 2 /* operand panels staged (and transposed) in LDS,  */
                            /* FP64 MFMA rank-4 updates                        */
#define MB_VARIANT_REGTILE 3 /* register tiles of 16-wide MFMA blocks read    */
                             /* straight from global memory (thin, flat and   */
                             /* small results)                                */

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

/* Host-only query: the kernel family (MB_VARIANT_DIRECT, _PACKED or _REGTILE)
 * that the plain calls select for this shape, or -1 for an illegal trans. */
int mb_dgemm_select(char transa, char transb, int m, int n, int k);

/* Host-only query: a static name of the kernel class the call would run
 * ("gemm_direct", "gemm_packed_tile64_k16", ...), for attributing profiles; the
 * scalar alpha/beta quick returns are not considered. */
const char *mb_dgemm_kernel_name(char transa, char transb, int m, int n, int k, int variant);

/*
 * Fortran-style aliases of mb_dgemm and mb_dpotrf (the dgemm_ calling form the
 * paper writes out in Sec. 2.1): every scalar argument -- trans and uplo
 * characters, sizes, leading dimensions, alpha, beta -- is passed by (host)
 * pointer, in the same positions, and the work goes to the null stream.
 * Matrices and info are device memory as in the plain calls.  A NULL scalar
 * pointer is an illegal value of that argument; otherwise the status and
 * semantics are those of mb_dgemm / mb_dpotrf.
 */
int mb_dgemm_(const char *transa, const char *transb, const int *m, const int *n, const int *k,
              const double *alpha, const double *A, const int *lda, const double *B,
              const int *ldb, const double *beta, double *C, const int *ldc);
int mb_dpotrf_(const char *uplo, const int *n, double *A, const int *lda, int *info);

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

/* ------------------------------------------------------------ backward --- */

/*
 * Reverse-mode derivatives (not in the paper, which has no differentiation;
 * they are built from its kernels: the dgemm adjoints are dgemm calls with
 * swapped transposition flags, the Cholesky adjoint uses the right-variant
 * triangular solve of Sec. 3.1.3 in 16 x 16 MFMA tiles).
 */

/*
 * For C = alpha*op(A)*op(B) + beta*C and the cotangent dC of the result:
 *   dA = alpha * dC * op(B)^T          (transa 'N'; A is m x k)
 *   dA = alpha * op(B) * dC^T          (transa 'T'; A is k x m)
 *   dB = alpha * op(A)^T * dC          (transb 'N'; B is k x n)
 *   dB = alpha * dC^T * op(A)          (transb 'T'; B is n x k)
 * (the cotangent of the input C is beta*dC and is not formed here).  dA and
 * dB are overwritten (not accumulated); either may be NULL to skip it.
 * Strided batches as in mb_dgemm_strided_batched; output strides must keep
 * instances disjoint.  Arguments: transa 1, transb 2, m 3, n 4, k 5, alpha 6,
 * A 7, lda 8, strideA 9, B 10, ldb 11, strideB 12, dC 13, lddc (>= max(1,m))
 * 14, stridedC 15, dA 16, ldda (>= max(1, rows of A)) 17, stridedA 18, dB 19,
 * lddb (>= max(1, rows of B)) 20, stridedB 21, batch 22, stream 23.
 * Device memory throughout; dA, dB must not overlap A, B or dC.
 */
int mb_dgemm_backward_strided_batched(char transa, char transb, int m, int n, int k, double alpha,
                                      const double *A, int lda, int64_t strideA, const double *B,
                                      int ldb, int64_t strideB, const double *dC, int lddc,
                                      int64_t stridedC, double *dA, int ldda, int64_t stridedA,
                                      double *dB, int lddb, int64_t stridedB, int batch,
                                      hipStream_t stream);

/*
 * Adjoint of the lower Cholesky factorization A = L*L^T: given the factor L
 * (lower triangle of an n x n array; the strict upper part is never read, so
 * the array mb_dpotrf wrote can be passed as is) and the cotangent Lbar of L
 * (lower triangle read), write the symmetric cotangent of A
 *   Abar = (S + S^T)/2,  S = L^{-T} Phi(L^T Lbar) L^{-1},
 * Phi taking the lower triangle with the diagonal halved, to all n x n
 * entries of Abar (the symmetric-gradient convention; <Abar, dA> is the
 * directional derivative for any symmetric dA).  n <= 304
 * (MB_ERR_UNSUPPORTED above).  Abar must not overlap L or Lbar; L must be a
 * successful factorization (nonzero diagonal).
 * Strided: n 1, L 2, ldl 3, strideL 4, Lbar 5, ldlb 6, strideLbar 7, Abar 8,
 * ldab 9, strideAbar 10 (>= ldab*(n-1)+n when batch > 1), batch 11, stream 12.
 * Pointer arrays: n 1, Larray 2, ldl 3, Lbararray 4, ldlb 5, Abararray 6,
 * ldab 7, batch 8, stream 9.
 */
int mb_dpotrf_l_backward_strided_batched(int n, const double *L, int ldl, int64_t strideL,
                                         const double *Lbar, int ldlb, int64_t strideLbar,
                                         double *Abar, int ldab, int64_t strideAbar, int batch,
                                         hipStream_t stream);
int mb_dpotrf_l_backward_batched(int n, const double *const *Larray, int ldl,
                                 const double *const *Lbararray, int ldlb,
                                 double *const *Abararray, int ldab, int batch, hipStream_t stream);

/*
 * LAPACK dlaset on a batch: the strictly upper ('U'), strictly lower ('L')
 * or all off-diagonal ('A') elements of each m x n matrix become alpha and
 * its diagonal beta; used to clear the triangle of a factor that dpotrf
 * leaves untouched.  Strided: uplo 1, m 2, n 3, alpha 4, beta 5, A 6, lda 7,
 * strideA 8, batch 9, stream 10.  Pointer arrays: uplo 1, m 2, n 3, alpha 4,
 * beta 5, Aarray 6, lda 7, batch 8, stream 9.
 */
int mb_dlaset_strided_batched(char uplo, int m, int n, double alpha, double beta, double *A,
                              int lda, int64_t strideA, int batch, hipStream_t stream);
int mb_dlaset_batched(char uplo, int m, int n, double alpha, double beta, double *const *Aarray,
                      int lda, int batch, hipStream_t stream);

/* ------------------------------------------------------ uneven batches --- */

/*
 * A batch of independent dgemm and dpotrf problems whose shapes all differ,
 * run by one persistent kernel.  The paper tunes one routine call at a time
 * and switches kernel variants by operand size (Sec. 2.4); it leaves batching
 * aside.  A plan applies the same size switch per problem: each dgemm is cut
 * into register tiles of one or two 16 x 16 MFMA blocks per side (chosen by
 * size), each dpotrf is one unit, units are ordered by a measured cost model
 * (longest first) and dealt to one work queue per XCD, and the persistent
 * grid drains the queues with atomic counters.  The launch is captured once
 * in a HIP graph.
 */
#define MB_OP_DGEMM 0
#define MB_OP_DPOTRF 1
#define MB_OP_DPOTRF_ADJOINT 2
#define MB_OP_DLASET 3

/*
 * One problem.  Every pointer is caller-owned DEVICE memory that must stay
 * valid (and must not be freed or moved) for the lifetime of the plan.
 *   dgemm  (op = MB_OP_DGEMM): C <= alpha*op(A)*op(B) + beta*C with the
 *          semantics, argument rules and quick returns of mb_dgemm; uplo and
 *          info are ignored.
 *   dpotrf (op = MB_OP_DPOTRF): the n x n matrix at C (leading dimension ldc)
 *          is factored in place as by mb_dpotrf('L'); *info receives the
 *          LAPACK info.  uplo must be 'L'/'l' ('U' is MB_ERR_UNSUPPORTED),
 *          n <= 304; transa, transb, m, k, alpha, beta, A, B are ignored.
 *   Cholesky adjoint (op = MB_OP_DPOTRF_ADJOINT): as
 *          mb_dpotrf_l_backward_strided_batched for one instance, with
 *          L = A (lda), Lbar = B (ldb), Abar = C (ldc), order n <= 304.
 *   dlaset (op = MB_OP_DLASET): as mb_dlaset_strided_batched for one m x n
 *          matrix C (ldc) with uplo, alpha, beta.
 * Every operand must span less than 4 GiB (MB_ERR_UNSUPPORTED otherwise).
 * Problems must not overlap each other's outputs.
 */
typedef struct mb_problem {
    int op;
    char transa, transb, uplo, reserved;
    int m, n, k;
    int lda, ldb, ldc;
    double alpha, beta;
    const double *A;
    const double *B;
    double *C;
    int *info;
} mb_problem;

typedef struct mb_plan mb_plan;

/*
 * Validate `problems` (host array of `count` >= 0 descriptors, read only
 * during the call), build the work queues in device memory on the current
 * device and capture the persistent launch in a HIP graph.  Allocates device
 * memory and synchronizes the device; *plan receives the handle.
 * Returns MB_OK; -1 (problems NULL with count > 0), -2 (count < 0), -3 (plan
 * NULL); MB_ERR_INVALID_PROBLEM or MB_ERR_UNSUPPORTED for the first failing
 * problem, whose index is stored to *bad_index when bad_index is not NULL;
 * MB_ERR_HIP.  Nothing is allocated when an error is returned.
 */
int mb_plan_create(const mb_problem *problems, int64_t count, mb_plan **plan,
                   int64_t *bad_index);

/*
 * Tuning overrides for mb_plan_create_ex (the autotuner's measurement
 * hooks; results never depend on them).  A negative field keeps the tuned
 * default.
 *   tile_two_min  a side of a dgemm register tile uses two 16-wide MFMA
 *                 blocks when that dimension of C exceeds this value.
 *   potrf_waves   waves of each 4-wave workgroup that start on the dpotrf /
 *                 Cholesky-adjoint class (0..4); the default follows that
 *                 class's share of the estimated work.
 */
typedef struct mb_plan_options {
    int tile_two_min;
    int potrf_waves;
} mb_plan_options;

/* mb_plan_create with tuning overrides (options may be NULL).  Positions:
 * problems 1, count 2, options 3 (-3: potrf_waves above 4), plan 4,
 * bad_index 5; mb_plan_create reports a NULL plan as -3. */
int mb_plan_create_ex(const mb_problem *problems, int64_t count, const mb_plan_options *options,
                      mb_plan **plan, int64_t *bad_index);

/* Execution modes of mb_plan_execute_mode. */
#define MB_PLAN_FUSED_GRAPH 0   /* the captured persistent launch (mb_plan_execute) */
#define MB_PLAN_FUSED 1         /* the same two kernels launched directly          */
#define MB_PLAN_GROUPED 2       /* one pointer-array batched call per distinct     */
                                /* (op, trans, uplo, m, n, k, ld, alpha, beta)     */
#define MB_PLAN_GROUPED_GRAPH 3 /* the grouped calls captured in a HIP graph      */
                                /* (captured at first use)                         */

/*
 * Run every problem of the plan on `stream` (enqueue only; no
 * synchronization).  Executions of one plan share its queue counters, so
 * they must be ordered (for example issued on one stream); the plan's device
 * must be current.  The grouped modes exist as the per-shape comparison for
 * the fused launch and give the same results (bitwise for dpotrf; dgemm
 * within rounding, the tile code differs).
 * Returns MB_OK, -1 (plan NULL), -2 (unknown mode), MB_ERR_HIP.
 */
int mb_plan_execute(mb_plan *plan, hipStream_t stream);
int mb_plan_execute_mode(mb_plan *plan, int mode, hipStream_t stream);

/*
 * Host-only statistics: out[i] for i < n (n <= 8) is
 *   0 problems, 1 work units, 2 dgemm groups, 3 groups of the other ops,
 *   4 persistent workgroups, 5 waves per CU, 6 problems with no work
 *   (quick returns), 7 total estimated cost in nanoseconds of wave time.
 * Returns MB_OK, -1 (plan NULL), -2 (out NULL with n > 0).
 */
int mb_plan_stats(const mb_plan *plan, int64_t *out, int n);

/* Wait for the plan's device, then free everything it owns.  NULL is a no-op. */
int mb_plan_destroy(mb_plan *plan);

/* ------------------------------------------------------ Riccati recursion --- */

/*
 * Batched BLAS dtrmm with side 'R', uplo 'L', trans 'N', diag 'N' (Sec. 3.1.4;
 * the dtrmm_rlnn of Sec. 5.2), in place:  B <= alpha * B * A  for each m x n
 * B and n x n lower-triangular A (its strictly upper part is never read).
 * alpha == 0 sets B to zero without reading A.  B must not overlap A.
 * Arguments: m 1, n 2, alpha 3, A 4, lda (>= max(1,n)) 5, strideA 6, B 7,
 * ldb (>= max(1,m)) 8, strideB (>= ldb*(n-1)+m when batch > 1) 9, batch 10,
 * stream 11.
 */
int mb_dtrmm_rlnn_strided_batched(int m, int n, double alpha, const double *A, int lda,
                                  int64_t strideA, double *B, int ldb, int64_t strideB, int batch,
                                  hipStream_t stream);

/*
 * Batched BLAS dsyrk with uplo 'L', trans 'N' (Sec. 3.1.2; the dsyrk_ln of
 * Sec. 5.2): the lower triangle of C <= alpha * A * A^T + beta * C for each
 * n x n C and n x k A; the strictly upper triangle of C is never touched.
 * BLAS scalar rules: beta == 0 does not read C; alpha == 0 or k == 0 does not
 * read A; with beta == 1 as well the call returns at once.  C must not
 * overlap A.  Arguments: n 1, k 2, alpha 3, A 4, lda (>= max(1,n)) 5,
 * strideA 6, beta 7, C 8, ldc (>= max(1,n)) 9, strideC (>= ldc*(n-1)+n when
 * batch > 1) 10, batch 11, stream 12.
 */
int mb_dsyrk_ln_strided_batched(int n, int k, double alpha, const double *A, int lda,
                                int64_t strideA, double beta, double *C, int ldc, int64_t strideC,
                                int batch, hipStream_t stream);

/*
 * Batched backward Riccati recursion in the factorized form of Sec. 5.2,
 * for independent problems with nx states, nu controls and horizon N
 * (m = nu + nx):
 *   LN   = chol(Q_N)                                         (lower)
 *   for n = N-1 down to 0:
 *     C_n  = BAt_n * Lc_{n+1}                (dtrmm_rlnn; Lc_N = LN)
 *     F_n  = chol(RSQ_n + C_n * C_n^T) = [Lambda_n 0; L_n Lc_n]
 *                                            (dsyrk_ln fused with dpotrf_l)
 *     Lc_n = F_n(nu:m, nu:m), the lower Cholesky factor of P_n
 * BAt_n = [B_n^T; A_n^T] is m x nx, RSQ_n = [R_n S_n; S_n^T Q_n] is m x m
 * symmetric (lower triangle read), Q_N is nx x nx (lower triangle read).  With
 * P = Lc_{n+1} Lc_{n+1}^T this is the Riccati update
 *   P_n = Q + A^T P A - (S^T + A^T P B)(R + B^T P B)^{-1}(S + B^T P A).
 * Layout: stage n of problem b of X starts at X + b*strideX + n*stageX,
 * column-major with leading dimension ldX.  Input stage strides may be 0
 * (time-invariant stages); inputs may be shared between problems.
 * Outputs: the lower triangles of F_n (m x m) and LN (nx x nx); their strictly
 * upper parts are never touched.  info (device, batch * (N+1) ints): entry
 * b*(N+1) + n is the dpotrf info of stage n of problem b, entry b*(N+1) + N
 * that of Q_N (LAPACK: 0, or the failing column + 1); a failed factorization
 * stops that problem's recursion, and the stages below it are not computed
 * (F untouched, info -1).  At a failing factorization only the columns before
 * the failing one hold factor values; the rest of that output is unspecified.
 * F may be RSQ itself (same pointer, ldf, stage and problem strides: in
 * place), and LN may be QN itself; otherwise outputs must not overlap inputs,
 * each other or the workspace.
 * work: device workspace of work_bytes bytes, private to the call while it
 * runs (calls that share one race).  Each wave of the kernel owns one slot of
 * 2 KiB * ceil(m/16) * ceil(nx/16) and takes problems w, w + W, ...; W is the
 * smallest of batch, the slots that fit in work_bytes and the waves the
 * device holds at once.  mb_riccati_workspace_size gives the size for the
 * largest W (one slot is enough for a correct, slower run).  Problems with
 * m <= 16, or whose C has at most 6 tiles of 16 x 16, keep C on chip and do
 * not touch the workspace (it is still validated).  m <= 304
 * (MB_ERR_UNSUPPORTED above).
 * Arguments: nx 1, nu 2, N 3, BAt 4, ldbat (>= max(1,m)) 5, stageBAt 6,
 * strideBAt 7, RSQ 8, ldrsq (>= max(1,m)) 9, stageRSQ 10, strideRSQ 11, QN 12,
 * ldq (>= max(1,nx)) 13, strideQ 14, F 15, ldf (>= max(1,m)) 16, stageF
 * (>= ldf*(m-1)+m when N > 1) 17, strideF (>= (N-1)*stageF + ldf*(m-1)+m
 * when batch > 1) 18, LN 19, ldl (>= max(1,nx)) 20, strideL
 * (>= ldl*(nx-1)+nx when batch > 1) 21, info 22, work 23, work_bytes (at
 * least one slot) 24, batch 25, stream 26.
 */
int mb_riccati_strided_batched(int nx, int nu, int N, const double *BAt, int ldbat,
                               int64_t stageBAt, int64_t strideBAt, const double *RSQ, int ldrsq,
                               int64_t stageRSQ, int64_t strideRSQ, const double *QN, int ldq,
                               int64_t strideQ, double *F, int ldf, int64_t stageF,
                               int64_t strideF, double *LN, int ldl, int64_t strideL, int *info,
                               void *work, size_t work_bytes, int batch, hipStream_t stream);

/*
 * Allocation-free variant of mb_riccati_strided_batched, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops
 * that forbid hipMalloc): the same recursion, results bit-identical to
 * mb_riccati_strided_batched, but the workspace slots come from a device
 * scratch array inside the library (64 MiB per device, held from the first
 * load of the library until the process ends) instead of a caller's buffer.
 * The call allocates nothing and never synchronizes.  The kernel's waves are
 * limited to the slots that fit in the scratch (64 MiB / the slot size of
 * mb_riccati_strided_batched), so shapes whose C does not stay on chip run
 * with fewer concurrent waves than a full-occupancy workspace allows.
 * Every call on one device shares that device's scratch: calls that overlap
 * in time on one device (different streams, different host threads) race;
 * calls ordered on one stream are safe, and nothing needs clearing between
 * them.  A shape whose single slot exceeds the scratch returns MB_ERR_SCRATCH
 * (no shape with nu + nx <= 304 does: the largest slot is 722 KiB).
 * Arguments and positions are those of mb_riccati_strided_batched without
 * work and work_bytes: batch is argument 23, stream 24.  MB_ERR_HIP when the
 * scratch address cannot be resolved or the launch fails.
 */
int mb_riccati_strided_batched_noalloc(int nx, int nu, int N, const double *BAt, int ldbat,
                                       int64_t stageBAt, int64_t strideBAt, const double *RSQ,
                                       int ldrsq, int64_t stageRSQ, int64_t strideRSQ,
                                       const double *QN, int ldq, int64_t strideQ, double *F,
                                       int ldf, int64_t stageF, int64_t strideF, double *LN,
                                       int ldl, int64_t strideL, int *info, int batch,
                                       hipStream_t stream);

/*
 * Workspace bytes for mb_riccati_strided_batched at full occupancy of the
 * current device: one slot per wave the device holds at once, at most batch
 * (at least one) slots.  Arguments: nx 1, nu 2, batch 3, bytes (host) 4;
 * MB_ERR_UNSUPPORTED when nx + nu > 304, MB_ERR_HIP on a failed device query.
 */
int mb_riccati_workspace_size(int nx, int nu, int batch, size_t *bytes);

/* ---------------------------------------------------------- ceilings --- */

/*
 * Measured FP64 compute ceilings (roofline support; not part of the BLAS
 * path).  Launches a register-only loop on `stream`: kind 0 = FP64 matrix
 * cores (v_mfma_f64_16x16x4, four independent chains per wave), kind 1 =
 * FP64 vector FMA (eight chains per lane); `blocks` workgroups of 256 threads
 * each run `iters` iterations and store one double per thread to `out`
 * (device, blocks * 256 doubles, caller-owned).  *flops (host) receives the
 * exact flop count of the launch; the caller times it (events on `stream`).
 * Arguments: kind 1, blocks 2, iters 3, out 4, flops 5 (illegal -> -position);
 * MB_ERR_HIP on a launch failure.
 */
int mb_ceiling_fp64(int kind, int blocks, int iters, double *out, double *flops,
                    hipStream_t stream);

/*
 * Measured HBM ceiling (roofline support; not part of the BLAS path).  One
 * streaming launch on `stream` over device buffers the caller owns, with
 * 16-byte non-temporal loads and stores and four loads in flight per thread:
 * kind 0 = read src[0, n) (one double per thread of the grid is stored to
 * `out`, blocks * 256 doubles), kind 1 = copy dst[0, n) = src[0, n), kind 2 =
 * three reads per write, dst[i] = src[i] + src[n + i] + src[2n + i] (src
 * holds 3n doubles).  `blocks` workgroups of 256 threads walk the buffer with
 * a grid stride.  *bytes (host) receives the bytes the launch must move
 * (8n, 16n, 32n); the caller times it.  Buffers must not overlap and must be
 * 16-byte aligned (torch allocations are).
 * Arguments: kind 1, src 2, dst (unused for kind 0) 3, n (> 0, even) 4,
 * blocks 5, out (kind 0) 6, bytes 7 (illegal -> -position); MB_ERR_HIP on a
 * launch failure.
 */
int mb_ceiling_hbm(int kind, const double *src, double *dst, int64_t n, int blocks, double *out,
                   double *bytes, hipStream_t stream);

/* ---------------------------------------------------------------- misc --- */

/* Static text for a status code (never NULL). */
const char *mb_status_string(int status);

/* Library version as major*10000 + minor*100 + patch. */
int mb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MI355BLAS_H */
