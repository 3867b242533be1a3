// mb_internal.h -- argument blocks, device helpers and launcher declarations
// shared by the gfx950 kernels and the host-side C ABI of mi355blas.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace mb {

// One batched dgemm call, already validated.  Instance b of X is
// Xarr[b] when Xarr != nullptr (pointer-array batch), else X + b*sX.
struct GemmArgs {
    int m, n, k;
    double alpha, beta;
    const double *A;
    const double *const *Aarr;
    int64_t sA;
    int lda;
    const double *B;
    const double *const *Barr;
    int64_t sB;
    int ldb;
    double *C;
    double *const *Carr;
    int64_t sC;
    int ldc;
    int batch;
};

// One batched lower-Cholesky call, already validated.
struct PotrfArgs {
    int n;
    double *A;
    double *const *Aarr;
    int64_t sA;
    int lda;
    int *info;
    int batch;
};

// One batched Cholesky-adjoint call, already validated.
struct PotrfAdjArgs {
    int n;
    const double *L;
    const double *const *Larr;
    int64_t sL;
    int ldl;
    const double *Lbar;
    const double *const *Lbararr;
    int64_t sLbar;
    int ldlb;
    double *Abar;
    double *const *Abararr;
    int64_t sAbar;
    int ldab;
    int batch;
};

// One batched dlaset call (uplo 0 = upper, 1 = lower, 2 = all), validated.
struct LasetArgs {
    int uplo, m, n;
    double alpha, beta;
    double *A;
    double *const *Aarr;
    int64_t sA;
    int lda;
    int batch;
};

// One batched dtrmm ('R','L','N','N': B <= alpha B A) call, already validated.
struct TrmmArgs {
    int m, n;
    double alpha;
    const double *A;
    int64_t sA;
    int lda;
    double *B;
    int64_t sB;
    int ldb;
    int batch;
};

// One batched dsyrk ('L','N': lower C <= alpha A A^T + beta C) call, validated.
struct SyrkArgs {
    int n, k;
    double alpha, beta;
    const double *A;
    int64_t sA;
    int lda;
    double *C;
    int64_t sC;
    int ldc;
    int batch;
};

// One batched Riccati recursion call, already validated.  Problem b, stage n
// of X is at X + b * sX + n * stX; info has N + 1 entries per problem.
struct RiccatiArgs {
    int nx, nu, N;
    const double *BAt;
    int64_t stBAt, sBAt;
    int ldbat;
    const double *RSQ;
    int64_t stRSQ, sRSQ;
    int ldrsq;
    const double *QN;
    int64_t sQ;
    int ldq;
    double *F;
    int64_t stF, sF;
    int ldf;
    double *LN;
    int64_t sL;
    int ldl;
    int *info;
    double *work;  // riccati_slot_doubles(nx, nu) doubles per wave
    int64_t batch;
};

typedef double d4 __attribute__((ext_vector_type(4)));

// Pointers known to address global memory.  Addresses that reach a kernel
// through memory (descriptor tables) are generic to the compiler, which then
// emits flat instructions; casting them keeps the global forms (scalar base +
// vector offset, no LDS-counter waits).
#define MB_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ MB_GLOBAL T *global_ptr(T *p)
{
    return (MB_GLOBAL T *)p;
}

// One unit of work of a fused uneven batch (plan.hip builds these, fused.hip
// runs them): a register tile of a dgemm, or a whole dpotrf.
//   kind < FUSED_POTRF: dgemm with trans code (kind & 3) = 2*ta + tb and a
//     register tile of TM = 1 + ((kind >> 2) & 1) by TN = 1 + (kind >> 3)
//     16 x 16 MFMA blocks whose first row / column are i0 / j0.  alpha == 0
//     or k == 0 is stored as alpha = 0, k = 0 (C = beta C).
//   kind == FUSED_POTRF: lower Cholesky of the n x n matrix at C (leading
//     dimension ldc), info to *info.
//   kind == FUSED_POTRF_ADJ, FUSED_LASET: see below.
// 96 bytes, so that a wave fetches one with a few scalar loads.
struct FusedTask {
    const double *A, *B;
    double *C;
    int *info;
    double alpha, beta;
    int m, n, k;
    int lda, ldb, ldc;
    int kind, i0, j0;
    int pad[3];
};
static_assert(sizeof(FusedTask) == 96, "FusedTask layout");
constexpr int FUSED_POTRF = 16;
constexpr int FUSED_POTRF_ADJ = 17;  // Cholesky adjoint: A = L, B = Lbar, C = Abar
constexpr int FUSED_LASET = 18;      // dlaset of columns j0 .. j0 + FUSED_LASET_COLS - 1 of C
                                     // (k = 0 upper, 1 lower, 2 all)
constexpr int FUSED_LASET_COLS = 64;
constexpr int kFusedWaves = 4;        // waves per workgroup of the fused kernel
constexpr int FUSED_XCDS = 8;         // XCDs of the device: one queue pair each
constexpr int FUSED_CLASSES = 2;      // queue class 0: dpotrf, 1: dgemm
constexpr int FUSED_QUEUES = FUSED_XCDS * FUSED_CLASSES;  // queue 2 x + class
constexpr int FUSED_CTR_STRIDE = 32;  // ints between queue counters (128 B)

struct FusedArgs {
    const FusedTask *tasks;
    const int *qoff;  // FUSED_QUEUES + 1 offsets into tasks
    int *counters;    // FUSED_QUEUES counters, FUSED_CTR_STRIDE apart
    int potrf_waves;  // waves per workgroup that start on the dpotrf class
};

__device__ __forceinline__ const double *inst_ptr(const double *base, const double *const *arr,
                                                  int64_t stride, int64_t b)
{
    return arr ? arr[b] : base + b * stride;
}
__device__ __forceinline__ double *inst_ptr(double *base, double *const *arr, int64_t stride,
                                            int64_t b)
{
    return arr ? arr[b] : base + b * stride;
}

// FP64 matrix-core step on one wave: D(16x16) += Aop(16x4) * Bop(4x16).
// Operand lanes: Aop[l%16][l/16] and Bop[l/16][l%16]; result register r of
// lane l is D[l/16 + 4*r][l%16] (rows interleaved across the registers).
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Make LDS writes of this wave visible to all of its lanes (single-wave
// groups use this instead of a workgroup barrier).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Make this wave's global stores visible to its own later global loads (from
// any lane).  The lanes of a wave share one CU and its vector L1, which the
// stores update on their way to L2, so a workgroup-scope release/acquire pair
// suffices: it waits until the stores have completed and needs no cache
// invalidation (an agent-scope acquire would also invalidate L2 lines).
__device__ __forceinline__ void wave_mem_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <bool WAVE_ONLY>
__device__ __forceinline__ void group_sync()
{
    if constexpr (WAVE_ONLY)
        wave_lds_sync();
    else
        __syncthreads();
}

// Workgroup b is dispatched to XCD b % 8; hand each XCD a contiguous range of
// logical work ids so that tiles of one instance share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblk)
{
    constexpr int NX = 8;
    const int per = nblk / NX;
    if (bid >= per * NX)
        return bid;
    return (bid % NX) * per + bid / NX;
}

// ---- launchers (host) -------------------------------------------------------
hipError_t launch_gemm_direct(bool ta, bool tb, const GemmArgs &a, hipStream_t s);
hipError_t launch_gemm_packed_config(int config, bool ta, bool tb, const GemmArgs &a,
                                     hipStream_t s);
hipError_t launch_gemm_scale(const GemmArgs &a, hipStream_t s);
// Register tiles of tm x tn (1 or 2) MFMA blocks; every instance must span
// less than 4 GiB per operand (32-bit offsets).
hipError_t launch_gemm_regtile(bool ta, bool tb, int tm, int tn, const GemmArgs &a,
                               hipStream_t s);
hipError_t launch_potrf_lower(const PotrfArgs &a, hipStream_t s);
hipError_t launch_fill_info(int *info, int batch, hipStream_t s);
hipError_t launch_potrf_adj(const PotrfAdjArgs &a, hipStream_t s);
hipError_t launch_laset(const LasetArgs &a, hipStream_t s);

// The packed configuration menu (gemm_packed.hip).
int packed_config_count();
const char *packed_config_name(int config);
int packed_config_wave_limit(int config);  // > 0: largest m, n of a WAVE shape; 0: any

// Fused persistent batch (fused.hip).
hipError_t launch_fused(const FusedArgs &a, int grid, hipStream_t s);
hipError_t fused_grid(int *grid, int *waves_per_cu);  // persistent grid for the current device
hipError_t launch_scatter_info(const int *src, int *const *dst, int count, hipStream_t s);
hipError_t launch_trmm_rlnn(const TrmmArgs &a, hipStream_t s);
hipError_t launch_syrk_ln(const SyrkArgs &a, hipStream_t s);
int64_t riccati_slot_doubles(int nx, int nu);  // workspace of one wave
hipError_t riccati_max_waves(int nx, int nu, int *waves);  // waves resident at once
hipError_t launch_riccati(const RiccatiArgs &a, int waves, hipStream_t s);
// Device scratch of the allocation-free Riccati entry point: the calling
// device's address of a file-scope array of RIC_SCRATCH_BYTES (resolved once
// per device; nothing is allocated).
constexpr size_t RIC_SCRATCH_BYTES = size_t(64) << 20;
hipError_t riccati_scratch(void **ptr, size_t *bytes);

// Validated dgemm / dpotrf launches used by the C ABI and by plans (api.hip):
// quick returns, size-class dispatch, launch.  Return an MB_ status.
int run_gemm(int ta, int tb, GemmArgs &a, int variant, int config, hipStream_t s);
int run_potrf(PotrfArgs &a, hipStream_t s);

// Name of the potrf kernel class for order n (profiling attribution).
const char *potrf_kernel_name(int n);

// Largest order handled by the register-resident Cholesky kernel.
constexpr int POTRF_MAX_N = 19 * 16;
// Largest order factored with whole rows in lanes (four instances per wave).
constexpr int POTRF_ROWS_MAX_N = 32;

}  // namespace mb
