// api.hip -- host side of the mi355blas C ABI: argument validation, quick
// returns, size-class dispatch (Sec. 2.4: a no-pack variant for very small
// operands, a packed variant above a measured switching point), launch.
//
// No call allocates memory, synchronizes or keeps mutable global state.
#include <limits.h>
#include <stdint.h>

#include "../../include/mi355blas.h"
#include "gemm_tuned.h"
#include "mb_internal.h"

namespace {

using mb::GemmArgs;
using mb::PotrfArgs;

int trans_code(char t)  // 0 = N, 1 = T, -1 = illegal
{
    switch (t) {
    case 'N': case 'n': return 0;
    case 'T': case 't': case 'C': case 'c': return 1;
    default: return -1;
    }
}

// Size-class dispatch from the measured table (gemm_tuned.h): the switch
// between the direct and the packed family and the packed tile configuration
// depend on the trans case and max(m, n, k) only -- never on the batch -- so a
// batch computes every instance exactly as the single call does.
struct Choice {
    int variant, config;
};

int dim_class(int mx)
{
    int e = 0;
    while (e < mb::kGemmTuneEntries - 1 && mx > mb::kGemmTuneMaxDim[e])
        ++e;
    return e;
}

int size_class(int m, int n, int k)
{
    int mx = m > n ? m : n;
    return dim_class(mx > k ? mx : k);
}

// The table entry for a shape: results with both sides above 16 use the
// square table (class of max(m, n, k)); thin (n <= 16), flat (m <= 16) and
// small results use the skinny tables, so that the choice follows the
// shape of C as the paper's variant switch does for rectangular matrices
// (Sec. 2.3.2, App. C).  Results of at most 4 x 4 have a table of their own:
// there one 16-wide MFMA tile is mostly padding and the direct kernel can
// win at any k, which the m, n <= 16 table (tuned on 8..16) would hide.
const int *table_entry(int ta, int tb, int m, int n, int k)
{
    const int tc = 2 * ta + tb;
    if (m > 16 && n > 16)
        return mb::kGemmTune[tc][size_class(m, n, k)];
    if (m <= 4 && n <= 4)
        return mb::kGemmSkinny[3][tc][dim_class(k)];
    if (m <= 16 && n <= 16)
        return mb::kGemmSkinny[0][tc][dim_class(k)];
    if (m <= 16)
        return mb::kGemmSkinny[1][tc][dim_class(n > k ? n : k)];
    return mb::kGemmSkinny[2][tc][dim_class(m > k ? m : k)];
}

// A WAVE configuration holds a whole instance: fall back to the first TILE
// configuration when the instance does not fit (non-square shapes).
int fit_config(int config, int m, int n)
{
    const int lim = mb::packed_config_wave_limit(config);
    if (lim > 0 && (m > lim || n > lim))
        return 3;  // tile64_k16
    return config;
}

Choice select(int ta, int tb, int m, int n, int k, int variant)
{
    const int *t = table_entry(ta, tb, m, n, k);
    Choice c;
    c.variant = (variant == MB_VARIANT_AUTO) ? t[0] : variant;
    int cfg = t[1];
    if (c.variant == MB_VARIANT_PACKED && cfg < 0) {
        // the table picks the direct family here: use the smallest packed shape that fits
        const int mx = m > n ? m : n;
        cfg = mx <= 16 ? 0 : (mx <= 32 ? 1 : 3);
    }
    c.config = (c.variant == MB_VARIANT_PACKED) ? fit_config(cfg, m, n) : -1;
    return c;
}

int select_variant(int ta, int tb, int m, int n, int k)
{
    return select(ta, tb, m, n, k, MB_VARIANT_AUTO).variant;
}

int to_status(hipError_t e) { return e == hipSuccess ? MB_OK : MB_ERR_HIP; }

// The register-tile kernels address an operand with 32-bit byte offsets.
bool regtile_fits(int ta, int tb, const GemmArgs &a)
{
    const int64_t lim = ((int64_t)1 << 32) / 8;
    const int64_t acols = ta ? a.m : a.k, bcols = tb ? a.k : a.n;
    return (int64_t)a.lda * acols < lim && (int64_t)a.ldb * bcols < lim &&
           (int64_t)a.ldc * a.n < lim;
}

// Shared validation of the dgemm scalar arguments; positions of lda/ldb/ldc
// differ between the call forms and are passed in.
int check_gemm(char transa, char transb, int m, int n, int k, int lda, int ldb, int ldc,
               int pos_lda, int pos_ldb, int pos_ldc)
{
    const int ta = trans_code(transa), tb = trans_code(transb);
    if (ta < 0) return -1;
    if (tb < 0) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0) return -5;
    const int arows = ta ? k : m, brows = tb ? n : k;
    if (lda < (arows > 1 ? arows : 1)) return -pos_lda;
    if (ldb < (brows > 1 ? brows : 1)) return -pos_ldb;
    if (ldc < (m > 1 ? m : 1)) return -pos_ldc;
    return MB_OK;
}

int gemm_strided(char transa, char transb, int m, int n, int k, double alpha, const double *A,
                 int lda, int64_t strideA, const double *B, int ldb, int64_t strideB, double beta,
                 double *C, int ldc, int64_t strideC, int batch, int variant, int pos_variant,
                 hipStream_t stream, int config = -1)
{
    int st = check_gemm(transa, transb, m, n, k, lda, ldb, ldc, 8, 11, 15);
    if (st != MB_OK)
        return st;
    if (strideA < 0) return -9;
    if (strideB < 0) return -12;
    if (strideC < 0) return -16;
    if (batch < 0) return -17;
    if (variant < MB_VARIANT_AUTO || variant > MB_VARIANT_REGTILE) return -pos_variant;
    if (batch > 1 && m > 0 && n > 0 && strideC < (int64_t)ldc * (n - 1) + m) return -16;
    const bool work = m > 0 && n > 0 && batch > 0 && !((alpha == 0.0 || k == 0) && beta == 1.0);
    if (work) {
        const bool reads_ab = alpha != 0.0 && k > 0;
        if (reads_ab && !A) return -7;
        if (reads_ab && !B) return -10;
        if (!C) return -14;
    }
    GemmArgs a{};
    a.m = m; a.n = n; a.k = k; a.alpha = alpha; a.beta = beta;
    a.A = A; a.sA = strideA; a.lda = lda;
    a.B = B; a.sB = strideB; a.ldb = ldb;
    a.C = C; a.sC = strideC; a.ldc = ldc;
    a.batch = batch;
    return mb::run_gemm(trans_code(transa), trans_code(transb), a, variant, config, stream);
}

int gemm_array(char transa, char transb, int m, int n, int k, double alpha,
               const double *const *Aarray, int lda, const double *const *Barray, int ldb,
               double beta, double *const *Carray, int ldc, int batch, int variant,
               int pos_variant, hipStream_t stream)
{
    int st = check_gemm(transa, transb, m, n, k, lda, ldb, ldc, 8, 10, 13);
    if (st != MB_OK)
        return st;
    if (batch < 0) return -14;
    if (variant < MB_VARIANT_AUTO || variant > MB_VARIANT_REGTILE) return -pos_variant;
    const bool work = m > 0 && n > 0 && batch > 0 && !((alpha == 0.0 || k == 0) && beta == 1.0);
    if (work) {
        const bool reads_ab = alpha != 0.0 && k > 0;
        if (reads_ab && !Aarray) return -7;
        if (reads_ab && !Barray) return -9;
        if (!Carray) return -12;
    }
    GemmArgs a{};
    a.m = m; a.n = n; a.k = k; a.alpha = alpha; a.beta = beta;
    a.Aarr = Aarray; a.lda = lda;
    a.Barr = Barray; a.ldb = ldb;
    a.Carr = Carray; a.ldc = ldc;
    a.batch = batch;
    return mb::run_gemm(trans_code(transa), trans_code(transb), a, variant, -1, stream);
}

int uplo_check(char uplo)  // 0 lower, 1 upper (unsupported), -1 illegal
{
    switch (uplo) {
    case 'L': case 'l': return 0;
    case 'U': case 'u': return 1;
    default: return -1;
    }
}

}  // namespace

namespace mb {

// variant: MB_VARIANT_*; config >= 0 forces a packed configuration.
int run_gemm(int ta, int tb, GemmArgs &a, int variant, int config, hipStream_t s)
{
    if (a.m == 0 || a.n == 0 || a.batch == 0)
        return MB_OK;
    if ((a.alpha == 0.0 || a.k == 0) && a.beta == 1.0)
        return MB_OK;
    if (a.alpha == 0.0 || a.k == 0)
        return to_status(mb::launch_gemm_scale(a, s));
    if (config >= 0)
        return to_status(mb::launch_gemm_packed_config(config, ta, tb, a, s));
    const Choice c = select(ta, tb, a.m, a.n, a.k, variant);
    if (c.variant == MB_VARIANT_DIRECT)
        return to_status(mb::launch_gemm_direct(ta, tb, a, s));
    if (c.variant == MB_VARIANT_REGTILE && regtile_fits(ta, tb, a))
        return to_status(mb::launch_gemm_regtile(ta, tb, a.m > 16 ? 2 : 1, a.n > 16 ? 2 : 1, a, s));
    if (c.variant == MB_VARIANT_REGTILE)  // an operand too large for 32-bit offsets
        return to_status(mb::launch_gemm_packed_config(3, ta, tb, a, s));
    return to_status(mb::launch_gemm_packed_config(c.config, ta, tb, a, s));
}

int run_potrf(PotrfArgs &a, hipStream_t s)
{
    if (a.batch == 0)
        return MB_OK;
    if (a.n == 0)
        return to_status(mb::launch_fill_info(a.info, a.batch, s));
    return to_status(mb::launch_potrf_lower(a, s));
}

}  // namespace mb

// Shared by the workspace and the allocation-free Riccati entry points; with
// noalloc the workspace is the library's device scratch and batch is
// argument 23 (work and work_bytes are not in that argument list).
static int riccati_call(int nx, int nu, int N, const double *BAt, int ldbat, int64_t stageBAt,
                        int64_t strideBAt, const double *RSQ, int ldrsq, int64_t stageRSQ,
                        int64_t strideRSQ, const double *QN, int ldq, int64_t strideQ, double *F,
                        int ldf, int64_t stageF, int64_t strideF, double *LN, int ldl,
                        int64_t strideL, int *info, void *work, size_t work_bytes, int batch,
                        hipStream_t stream, bool noalloc)
{
    const int m = nx + nu;
    const int64_t span_f = m > 0 ? (int64_t)ldf * (m - 1) + m : 0;
    if (nx < 0) return -1;
    if (nu < 0) return -2;
    if (N < 0) return -3;
    if (ldbat < std::max(1, m)) return -5;
    if (stageBAt < 0) return -6;
    if (strideBAt < 0) return -7;
    if (ldrsq < std::max(1, m)) return -9;
    if (stageRSQ < 0) return -10;
    if (strideRSQ < 0) return -11;
    if (ldq < std::max(1, nx)) return -13;
    if (strideQ < 0) return -14;
    if (ldf < std::max(1, m)) return -16;
    if (stageF < 0 || (N > 1 && stageF < span_f)) return -17;
    if (strideF < 0 || (batch > 1 && N > 0 && strideF < (int64_t)(N - 1) * stageF + span_f))
        return -18;
    if (ldl < std::max(1, nx)) return -20;
    if (strideL < 0 || (batch > 1 && nx > 0 && strideL < (int64_t)ldl * (nx - 1) + nx))
        return -21;
    if (batch < 0) return noalloc ? -23 : -25;
    if (m > mb::POTRF_MAX_N) return MB_ERR_UNSUPPORTED;
    if (batch == 0)
        return MB_OK;
    if (!BAt && N > 0 && m > 0 && nx > 0) return -4;
    if (!RSQ && N > 0 && m > 0) return -8;
    if (!QN && nx > 0) return -12;
    if (!F && N > 0 && m > 0) return -15;
    if (!LN && nx > 0) return -19;
    if (!info) return -22;
    const int64_t slot = mb::riccati_slot_doubles(nx, nu);
    if (noalloc && slot > 0) {
        // the file-scope device scratch stands in for the caller's workspace
        const hipError_t se = mb::riccati_scratch(&work, &work_bytes);
        if (se != hipSuccess)
            return MB_ERR_HIP;
        if ((size_t)slot * sizeof(double) > work_bytes)
            return MB_ERR_SCRATCH;
    }
    const int64_t slots = slot > 0 ? (int64_t)(work_bytes / ((size_t)slot * sizeof(double))) : batch;
    if (slot > 0 && !work) return -23;
    if (slots < 1) return -24;
    int waves = 0;
    hipError_t e = mb::riccati_max_waves(nx, nu, &waves);
    if (e != hipSuccess)
        return MB_ERR_HIP;
    waves = (int)std::min<int64_t>(std::min<int64_t>(waves, slots), batch);
    mb::RiccatiArgs a{};
    a.nx = nx; a.nu = nu; a.N = N;
    a.BAt = BAt; a.stBAt = stageBAt; a.sBAt = strideBAt; a.ldbat = ldbat;
    a.RSQ = RSQ; a.stRSQ = stageRSQ; a.sRSQ = strideRSQ; a.ldrsq = ldrsq;
    a.QN = QN; a.sQ = strideQ; a.ldq = ldq;
    a.F = F; a.stF = stageF; a.sF = strideF; a.ldf = ldf;
    a.LN = LN; a.sL = strideL; a.ldl = ldl;
    a.info = info;
    a.work = (double *)work;
    a.batch = batch;
    return to_status(mb::launch_riccati(a, waves, stream));
}

extern "C" {

int mb_dgemm(char transa, char transb, int m, int n, int k, double alpha, const double *A,
             int lda, const double *B, int ldb, double beta, double *C, int ldc,
             hipStream_t stream)
{
    int st = check_gemm(transa, transb, m, n, k, lda, ldb, ldc, 8, 10, 13);
    if (st != MB_OK)
        return st;
    const bool work = m > 0 && n > 0 && !((alpha == 0.0 || k == 0) && beta == 1.0);
    if (work) {
        const bool reads_ab = alpha != 0.0 && k > 0;
        if (reads_ab && !A) return -7;
        if (reads_ab && !B) return -9;
        if (!C) return -12;
    }
    GemmArgs a{};
    a.m = m; a.n = n; a.k = k; a.alpha = alpha; a.beta = beta;
    a.A = A; a.lda = lda; a.B = B; a.ldb = ldb; a.C = C; a.ldc = ldc;
    a.batch = 1;
    return mb::run_gemm(trans_code(transa), trans_code(transb), a, MB_VARIANT_AUTO, -1, stream);
}

int mb_dgemm_strided_batched(char transa, char transb, int m, int n, int k, double alpha,
                             const double *A, int lda, int64_t strideA, const double *B, int ldb,
                             int64_t strideB, double beta, double *C, int ldc, int64_t strideC,
                             int batch, hipStream_t stream)
{
    return gemm_strided(transa, transb, m, n, k, alpha, A, lda, strideA, B, ldb, strideB, beta,
                        C, ldc, strideC, batch, MB_VARIANT_AUTO, 0, stream);
}

int mb_dgemm_strided_batched_ex(char transa, char transb, int m, int n, int k, double alpha,
                                const double *A, int lda, int64_t strideA, const double *B,
                                int ldb, int64_t strideB, double beta, double *C, int ldc,
                                int64_t strideC, int batch, int variant, hipStream_t stream)
{
    return gemm_strided(transa, transb, m, n, k, alpha, A, lda, strideA, B, ldb, strideB, beta,
                        C, ldc, strideC, batch, variant, 18, stream);
}

int mb_dgemm_strided_batched_config(char transa, char transb, int m, int n, int k,
                                    double alpha, const double *A, int lda, int64_t strideA,
                                    const double *B, int ldb, int64_t strideB, double beta,
                                    double *C, int ldc, int64_t strideC, int batch, int config,
                                    hipStream_t stream)
{
    if (config < 0 || config >= mb::packed_config_count())
        return -18;
    const int lim = mb::packed_config_wave_limit(config);
    if (lim > 0 && (m > lim || n > lim))
        return MB_ERR_UNSUPPORTED;
    return gemm_strided(transa, transb, m, n, k, alpha, A, lda, strideA, B, ldb, strideB, beta,
                        C, ldc, strideC, batch, MB_VARIANT_PACKED, 18, stream, config);
}

int mb_dgemm_config_count(void) { return mb::packed_config_count(); }

const char *mb_dgemm_config_name(int config) { return mb::packed_config_name(config); }

int mb_dgemm_config_max_mn(int config)
{
    if (config < 0 || config >= mb::packed_config_count())
        return -1;
    const int lim = mb::packed_config_wave_limit(config);
    return lim > 0 ? lim : INT_MAX;
}

int mb_dgemm_batched(char transa, char transb, int m, int n, int k, double alpha,
                     const double *const *Aarray, int lda, const double *const *Barray, int ldb,
                     double beta, double *const *Carray, int ldc, int batch, hipStream_t stream)
{
    return gemm_array(transa, transb, m, n, k, alpha, Aarray, lda, Barray, ldb, beta, Carray, ldc,
                      batch, MB_VARIANT_AUTO, 0, stream);
}

int mb_dgemm_batched_ex(char transa, char transb, int m, int n, int k, double alpha,
                        const double *const *Aarray, int lda, const double *const *Barray,
                        int ldb, double beta, double *const *Carray, int ldc, int batch,
                        int variant, hipStream_t stream)
{
    return gemm_array(transa, transb, m, n, k, alpha, Aarray, lda, Barray, ldb, beta, Carray, ldc,
                      batch, variant, 15, stream);
}

int mb_dgemm_select(char transa, char transb, int m, int n, int k)
{
    const int ta = trans_code(transa), tb = trans_code(transb);
    if (ta < 0 || tb < 0)
        return -1;
    return select_variant(ta, tb, m, n, k);
}

const char *mb_dgemm_kernel_name(char transa, char transb, int m, int n, int k, int variant)
{
    const int ta = trans_code(transa), tb = trans_code(transb);
    if (ta < 0 || tb < 0 || m < 0 || n < 0 || k < 0)
        return "illegal";
    if (m == 0 || n == 0)
        return "none";
    if (k == 0)
        return "gemm_scale";
    const Choice c = select(ta, tb, m, n, k, variant);
    if (c.variant == MB_VARIANT_DIRECT)
        return "gemm_direct";
    if (c.variant == MB_VARIANT_REGTILE) {
        static const char *names[4] = {"gemm_regtile_t11", "gemm_regtile_t21", "gemm_regtile_t12",
                                       "gemm_regtile_t22"};
        return names[(m > 16 ? 1 : 0) + (n > 16 ? 2 : 0)];
    }
    return mb::packed_config_name(c.config);
}

const char *mb_dpotrf_kernel_name(int n)
{
    if (n < 0 || n > mb::POTRF_MAX_N)
        return "unsupported";
    return mb::potrf_kernel_name(n);
}

int mb_dpotrf(char uplo, int n, double *A, int lda, int *info, hipStream_t stream)
{
    const int u = uplo_check(uplo);
    if (u < 0) return -1;
    if (n < 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (u == 1) return MB_ERR_UNSUPPORTED;
    if (n > mb::POTRF_MAX_N) return MB_ERR_UNSUPPORTED;
    if (n > 0 && !A) return -3;
    if (!info) return -5;
    PotrfArgs a{};
    a.n = n; a.A = A; a.lda = lda; a.info = info; a.batch = 1;
    return mb::run_potrf(a, stream);
}

int mb_dpotrf_strided_batched(char uplo, int n, double *A, int lda, int64_t strideA, int *info,
                              int batch, hipStream_t stream)
{
    const int u = uplo_check(uplo);
    if (u < 0) return -1;
    if (n < 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (strideA < 0) return -5;
    if (batch < 0) return -7;
    if (batch > 1 && n > 0 && strideA < (int64_t)lda * (n - 1) + n) return -5;
    if (u == 1) return MB_ERR_UNSUPPORTED;
    if (n > mb::POTRF_MAX_N) return MB_ERR_UNSUPPORTED;
    if (batch > 0 && n > 0 && !A) return -3;
    if (batch > 0 && !info) return -6;
    PotrfArgs a{};
    a.n = n; a.A = A; a.sA = strideA; a.lda = lda; a.info = info; a.batch = batch;
    return mb::run_potrf(a, stream);
}

int mb_dpotrf_batched(char uplo, int n, double *const *Aarray, int lda, int *info, int batch,
                      hipStream_t stream)
{
    const int u = uplo_check(uplo);
    if (u < 0) return -1;
    if (n < 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (batch < 0) return -6;
    if (u == 1) return MB_ERR_UNSUPPORTED;
    if (n > mb::POTRF_MAX_N) return MB_ERR_UNSUPPORTED;
    if (batch > 0 && n > 0 && !Aarray) return -3;
    if (batch > 0 && !info) return -5;
    PotrfArgs a{};
    a.n = n; a.Aarr = Aarray; a.lda = lda; a.info = info; a.batch = batch;
    return mb::run_potrf(a, stream);
}

int mb_dgemm_backward_strided_batched(char transa, char transb, int m, int n, int k, double alpha,
                                      const double *A, int lda, int64_t strideA, const double *B,
                                      int ldb, int64_t strideB, const double *dC, int lddc,
                                      int64_t stridedC, double *dA, int ldda, int64_t stridedA,
                                      double *dB, int lddb, int64_t stridedB, int batch,
                                      hipStream_t stream)
{
    const int ta = trans_code(transa), tb = trans_code(transb);
    if (ta < 0) return -1;
    if (tb < 0) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0) return -5;
    const int arows = ta ? k : m, acols = ta ? m : k;
    const int brows = tb ? n : k, bcols = tb ? k : n;
    if (lda < (arows > 1 ? arows : 1)) return -8;
    if (strideA < 0) return -9;
    if (ldb < (brows > 1 ? brows : 1)) return -11;
    if (strideB < 0) return -12;
    if (lddc < (m > 1 ? m : 1)) return -14;
    if (stridedC < 0) return -15;
    if (ldda < (arows > 1 ? arows : 1)) return -17;
    if (stridedA < 0 || (dA && batch > 1 && arows > 0 && acols > 0 &&
                         stridedA < (int64_t)ldda * (acols - 1) + arows))
        return -18;
    if (lddb < (brows > 1 ? brows : 1)) return -20;
    if (stridedB < 0 || (dB && batch > 1 && brows > 0 && bcols > 0 &&
                         stridedB < (int64_t)lddb * (bcols - 1) + brows))
        return -21;
    if (batch < 0) return -22;
    if (batch == 0)
        return MB_OK;
    const bool grad_a = dA && arows > 0 && acols > 0;
    const bool grad_b = dB && brows > 0 && bcols > 0;
    const bool reads = alpha != 0.0 && m > 0 && n > 0 && k > 0;
    if (reads && grad_a && (!dC || !B)) return !dC ? -13 : -10;
    if (reads && grad_b && (!dC || !A)) return !dC ? -13 : -7;
    const char nt[2] = {'N', 'T'};
    int st = MB_OK;
    // dA = alpha dC op(B)^T ('N' A) or alpha op(B) dC^T ('T' A)
    if (grad_a) {
        if (!ta)
            st = gemm_strided('N', nt[1 - tb], m, k, n, alpha, dC, lddc, stridedC, B, ldb,
                              strideB, 0.0, dA, ldda, stridedA, batch, MB_VARIANT_AUTO, 0, stream);
        else
            st = gemm_strided(nt[tb], 'T', k, m, n, alpha, B, ldb, strideB, dC, lddc, stridedC,
                              0.0, dA, ldda, stridedA, batch, MB_VARIANT_AUTO, 0, stream);
        if (st != MB_OK)
            return st < 0 && st > -64 ? MB_ERR_HIP : st;
    }
    // dB = alpha op(A)^T dC ('N' B) or alpha dC^T op(A) ('T' B)
    if (grad_b) {
        if (!tb)
            st = gemm_strided(nt[1 - ta], 'N', k, n, m, alpha, A, lda, strideA, dC, lddc,
                              stridedC, 0.0, dB, lddb, stridedB, batch, MB_VARIANT_AUTO, 0, stream);
        else
            st = gemm_strided('T', nt[ta], n, k, m, alpha, dC, lddc, stridedC, A, lda, strideA,
                              0.0, dB, lddb, stridedB, batch, MB_VARIANT_AUTO, 0, stream);
        if (st != MB_OK)
            return st < 0 && st > -64 ? MB_ERR_HIP : st;
    }
    return MB_OK;
}

int mb_dpotrf_l_backward_strided_batched(int n, const double *L, int ldl, int64_t strideL,
                                         const double *Lbar, int ldlb, int64_t strideLbar,
                                         double *Abar, int ldab, int64_t strideAbar, int batch,
                                         hipStream_t stream)
{
    if (n < 0) return -1;
    if (ldl < (n > 1 ? n : 1)) return -3;
    if (strideL < 0) return -4;
    if (ldlb < (n > 1 ? n : 1)) return -6;
    if (strideLbar < 0) return -7;
    if (ldab < (n > 1 ? n : 1)) return -9;
    if (strideAbar < 0 || (batch > 1 && n > 0 && strideAbar < (int64_t)ldab * (n - 1) + n))
        return -10;
    if (batch < 0) return -11;
    if (n > mb::POTRF_MAX_N) return MB_ERR_UNSUPPORTED;
    if (n == 0 || batch == 0)
        return MB_OK;
    if (!L) return -2;
    if (!Lbar) return -5;
    if (!Abar) return -8;
    mb::PotrfAdjArgs a{};
    a.n = n;
    a.L = L; a.sL = strideL; a.ldl = ldl;
    a.Lbar = Lbar; a.sLbar = strideLbar; a.ldlb = ldlb;
    a.Abar = Abar; a.sAbar = strideAbar; a.ldab = ldab;
    a.batch = batch;
    return to_status(mb::launch_potrf_adj(a, stream));
}

int mb_dpotrf_l_backward_batched(int n, const double *const *Larray, int ldl,
                                 const double *const *Lbararray, int ldlb,
                                 double *const *Abararray, int ldab, int batch, hipStream_t stream)
{
    if (n < 0) return -1;
    if (ldl < (n > 1 ? n : 1)) return -3;
    if (ldlb < (n > 1 ? n : 1)) return -5;
    if (ldab < (n > 1 ? n : 1)) return -7;
    if (batch < 0) return -8;
    if (n > mb::POTRF_MAX_N) return MB_ERR_UNSUPPORTED;
    if (n == 0 || batch == 0)
        return MB_OK;
    if (!Larray) return -2;
    if (!Lbararray) return -4;
    if (!Abararray) return -6;
    mb::PotrfAdjArgs a{};
    a.n = n;
    a.Larr = Larray; a.ldl = ldl;
    a.Lbararr = Lbararray; a.ldlb = ldlb;
    a.Abararr = Abararray; a.ldab = ldab;
    a.batch = batch;
    return to_status(mb::launch_potrf_adj(a, stream));
}

static int laset_uplo(char u)
{
    switch (u) {
    case 'U': case 'u': return 0;
    case 'L': case 'l': return 1;
    case 'A': case 'a': return 2;
    default: return -1;
    }
}

int mb_dlaset_strided_batched(char uplo, int m, int n, double alpha, double beta, double *A,
                              int lda, int64_t strideA, int batch, hipStream_t stream)
{
    const int u = laset_uplo(uplo);
    if (u < 0) return -1;
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (lda < (m > 1 ? m : 1)) return -7;
    if (strideA < 0 || (batch > 1 && m > 0 && n > 0 && strideA < (int64_t)lda * (n - 1) + m))
        return -8;
    if (batch < 0) return -9;
    if (m == 0 || n == 0 || batch == 0)
        return MB_OK;
    if (!A) return -6;
    mb::LasetArgs a{};
    a.uplo = u; a.m = m; a.n = n; a.alpha = alpha; a.beta = beta;
    a.A = A; a.sA = strideA; a.lda = lda; a.batch = batch;
    return to_status(mb::launch_laset(a, stream));
}

int mb_dlaset_batched(char uplo, int m, int n, double alpha, double beta, double *const *Aarray,
                      int lda, int batch, hipStream_t stream)
{
    const int u = laset_uplo(uplo);
    if (u < 0) return -1;
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (lda < (m > 1 ? m : 1)) return -7;
    if (batch < 0) return -8;
    if (m == 0 || n == 0 || batch == 0)
        return MB_OK;
    if (!Aarray) return -6;
    mb::LasetArgs a{};
    a.uplo = u; a.m = m; a.n = n; a.alpha = alpha; a.beta = beta;
    a.Aarr = Aarray; a.lda = lda; a.batch = batch;
    return to_status(mb::launch_laset(a, stream));
}

int mb_dgemm_(const char *transa, const char *transb, const int *m, const int *n, const int *k,
              const double *alpha, const double *A, const int *lda, const double *B,
              const int *ldb, const double *beta, double *C, const int *ldc)
{
    // every scalar is read through its pointer; a missing one is illegal
    if (!transa) return -1;
    if (!transb) return -2;
    if (!m) return -3;
    if (!n) return -4;
    if (!k) return -5;
    if (!alpha) return -6;
    if (!lda) return -8;
    if (!ldb) return -10;
    if (!beta) return -11;
    if (!ldc) return -13;
    return mb_dgemm(*transa, *transb, *m, *n, *k, *alpha, A, *lda, B, *ldb, *beta, C, *ldc,
                    nullptr);
}

int mb_dpotrf_(const char *uplo, const int *n, double *A, const int *lda, int *info)
{
    if (!uplo) return -1;
    if (!n) return -2;
    if (!lda) return -4;
    return mb_dpotrf(*uplo, *n, A, *lda, info, nullptr);
}

int mb_dtrmm_rlnn_strided_batched(int m, int n, double alpha, const double *A, int lda,
                                  int64_t strideA, double *B, int ldb, int64_t strideB, int batch,
                                  hipStream_t stream)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (lda < std::max(1, n)) return -5;
    if (strideA < 0) return -6;
    if (ldb < std::max(1, m)) return -8;
    if (strideB < 0 || (batch > 1 && m > 0 && n > 0 && strideB < (int64_t)ldb * (n - 1) + m))
        return -9;
    if (batch < 0) return -10;
    if (m == 0 || n == 0 || batch == 0)
        return MB_OK;
    if (!A && alpha != 0.0) return -4;
    if (!B) return -7;
    mb::TrmmArgs a{};
    a.m = m; a.n = n; a.alpha = alpha;
    a.A = A; a.sA = strideA; a.lda = lda;
    a.B = B; a.sB = strideB; a.ldb = ldb;
    a.batch = batch;
    return to_status(mb::launch_trmm_rlnn(a, stream));
}

int mb_dsyrk_ln_strided_batched(int n, int k, double alpha, const double *A, int lda,
                                int64_t strideA, double beta, double *C, int ldc, int64_t strideC,
                                int batch, hipStream_t stream)
{
    if (n < 0) return -1;
    if (k < 0) return -2;
    if (lda < std::max(1, n)) return -5;
    if (strideA < 0) return -6;
    if (ldc < std::max(1, n)) return -9;
    if (strideC < 0 || (batch > 1 && n > 0 && strideC < (int64_t)ldc * (n - 1) + n)) return -10;
    if (batch < 0) return -11;
    if (n == 0 || batch == 0 || ((alpha == 0.0 || k == 0) && beta == 1.0))
        return MB_OK;
    if (!A && alpha != 0.0 && k > 0) return -4;
    if (!C) return -8;
    mb::SyrkArgs a{};
    a.n = n; a.k = k; a.alpha = (k == 0) ? 0.0 : alpha; a.beta = beta;
    a.A = A; a.sA = strideA; a.lda = lda;
    a.C = C; a.sC = strideC; a.ldc = ldc;
    a.batch = batch;
    return to_status(mb::launch_syrk_ln(a, stream));
}

int mb_riccati_workspace_size(int nx, int nu, int batch, size_t *bytes)
{
    if (nx < 0) return -1;
    if (nu < 0) return -2;
    if (batch < 0) return -3;
    if (!bytes) return -4;
    if (nx + nu > mb::POTRF_MAX_N) return MB_ERR_UNSUPPORTED;
    int waves = 0;
    const hipError_t e = mb::riccati_max_waves(nx, nu, &waves);
    if (e != hipSuccess)
        return MB_ERR_HIP;
    const int64_t w = std::max<int64_t>(1, std::min<int64_t>(batch, waves));
    *bytes = (size_t)(w * mb::riccati_slot_doubles(nx, nu) * (int64_t)sizeof(double));
    return MB_OK;
}

int mb_riccati_strided_batched(int nx, int nu, int N, const double *BAt, int ldbat,
                               int64_t stageBAt, int64_t strideBAt, const double *RSQ, int ldrsq,
                               int64_t stageRSQ, int64_t strideRSQ, const double *QN, int ldq,
                               int64_t strideQ, double *F, int ldf, int64_t stageF,
                               int64_t strideF, double *LN, int ldl, int64_t strideL, int *info,
                               void *work, size_t work_bytes, int batch, hipStream_t stream)
{
    return riccati_call(nx, nu, N, BAt, ldbat, stageBAt, strideBAt, RSQ, ldrsq, stageRSQ,
                        strideRSQ, QN, ldq, strideQ, F, ldf, stageF, strideF, LN, ldl, strideL,
                        info, work, work_bytes, batch, stream, false);
}

int mb_riccati_strided_batched_noalloc(int nx, int nu, int N, const double *BAt, int ldbat,
                                       int64_t stageBAt, int64_t strideBAt, const double *RSQ,
                                       int ldrsq, int64_t stageRSQ, int64_t strideRSQ,
                                       const double *QN, int ldq, int64_t strideQ, double *F,
                                       int ldf, int64_t stageF, int64_t strideF, double *LN,
                                       int ldl, int64_t strideL, int *info, int batch,
                                       hipStream_t stream)
{
    return riccati_call(nx, nu, N, BAt, ldbat, stageBAt, strideBAt, RSQ, ldrsq, stageRSQ,
                        strideRSQ, QN, ldq, strideQ, F, ldf, stageF, strideF, LN, ldl, strideL,
                        info, nullptr, 0, batch, stream, true);
}

const char *mb_status_string(int status)
{
    if (status == MB_OK) return "success";
    if (status == MB_ERR_HIP) return "HIP runtime or launch failure";
    if (status == MB_ERR_UNSUPPORTED) return "unsupported argument combination";
    if (status == MB_ERR_INVALID_PROBLEM) return "a plan problem failed validation";
    if (status == MB_ERR_SCRATCH)
        return "the problem needs more device scratch than the allocation-free entry point holds";
    if (status < 0 && status > -64) return "illegal value of argument -status";
    return "unknown status";
}

int mb_version(void) { return 100; }

}  // extern "C"
