// fused.hip -- one persistent kernel for an uneven batch of dgemm and dpotrf
// problems of mixed sizes.
//
// The paper switches between kernel variants by operand size (Sec. 2.4) but
// leaves batching aside; a batch whose problems all differ in shape cannot be
// served by per-shape launches without paying one launch per shape.  Here a
// plan (plan.hip) turns the batch into work units -- one register tile of a
// dgemm, or one whole dpotrf -- sorted by estimated cost and dealt to one
// queue per XCD.  Every wave of the persistent grid is an independent worker:
// it claims the next unit of its XCD's queue with one atomic increment, runs
// it, and moves on to the other queues once its own is empty, so the grid
// drains every queue whatever the dispatch order.
//
// dgemm units are TM x TN tiles of 16 x 16 FP64 MFMA blocks computed straight
// from global memory: within one wave the operand fragments of a 16-deep k
// chunk partition the A and B panels exactly (lane (g, i) holds k = kk + 4g +
// s, s = 0..3, of row i), so there is no redundant load to share through LDS
// and no LDS traffic or barrier at all.  As in the batched kernels the MFMA
// takes op(B) as its left operand and accumulates C^T, so a lane owns whole
// rows of C and the epilogue stores are coalesced along columns.  dpotrf units
// run the batched kernel's per-wave factorization (one block column at a
// time, which keeps the register budget of the fused kernel low).
#include "potrf_wave.h"

namespace mb {

// op(A)[i][k] lives at A[i + k lda] ('N') or A[k + i lda] ('T'); op(B)[k][j]
// at B[k + j ldb] ('N') or B[j + k ldb] ('T').  Rows of op(A) past m and
// columns of op(B) past n read a clamped in-range address instead: entry
// (i, j) of the product depends on row i of op(A) and column j of op(B) only,
// so the padded lanes affect just the C entries that are never stored, and no
// load is predicated off.  The k tail chunk clamps k the same way but must
// zero what it read, since every output sums over k.
//
// Addresses are a wave-uniform base (advanced by one k chunk per step) plus a
// loop-invariant 32-bit byte offset per lane, which maps onto the
// scalar-base + vector-offset form of the global loads and keeps the address
// registers to one per operand fragment (plans check that every operand spans
// less than 4 GiB).
__device__ __forceinline__ MB_GLOBAL double &at(double *base, uint32_t byte_off)
{
    return *(MB_GLOBAL double *)((MB_GLOBAL char *)global_ptr(base) + byte_off);
}
__device__ __forceinline__ const MB_GLOBAL double &at(const double *base, uint32_t byte_off)
{
    return *(const MB_GLOBAL double *)((const MB_GLOBAL char *)global_ptr(base) + byte_off);
}

// Wave-uniform copies in scalar registers (the descriptor is read with
// vector loads -- the kernel writes memory, so the compiler cannot prove it
// read-only -- and would otherwise stay in vector registers, which rules out
// the scalar-base address form).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t uni(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ double uni(double x)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = uni((uint32_t)b), hi = uni((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T *uni(T *p)
{
    const uint64_t b = (uint64_t)p;
    const uint32_t lo = uni((uint32_t)b), hi = uni((uint32_t)(b >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}

template <bool TA, bool TB, int TM, int TN>
__device__ __forceinline__ void regtile(const FusedDesc &d, uint32_t tile, int lane)
{
    const int lr = lane & 15, lg = lane >> 4;
    const uint32_t tiles_m = uni((uint32_t)d.tiles_m);
    const int tm = (int)(tile % tiles_m);
    const int tn = (int)(tile / tiles_m);
    const int i0 = tm * 16 * TM, j0 = tn * 16 * TN;
    const int m = uni(d.m), n = uni(d.n), K = uni(d.k);
    const uint32_t lda = uni((uint32_t)d.lda), ldb = uni((uint32_t)d.ldb),
                   ldc = uni((uint32_t)d.ldc);
    const uint32_t ska = TA ? 1u : lda;  // element step along k in A
    const uint32_t skb = TB ? ldb : 1u;  // element step along k in B

    // per-lane element offset of (row, k = 4 lg) of each fragment
    uint32_t oa[TM], ob[TN];
#pragma unroll
    for (int ti = 0; ti < TM; ++ti) {
        const int i = i0 + ti * 16 + lr;
        const uint32_t ic = (uint32_t)(i < m ? i : m - 1);
        oa[ti] = (TA ? ic * lda : ic) + (uint32_t)(4 * lg) * ska;
    }
#pragma unroll
    for (int tj = 0; tj < TN; ++tj) {
        const int j = j0 + tj * 16 + lr;
        const uint32_t jc = (uint32_t)(j < n ? j : n - 1);
        ob[tj] = (TB ? jc : jc * ldb) + (uint32_t)(4 * lg) * skb;
    }

    const double alpha = uni(d.alpha), beta = uni(d.beta);
    double *C = uni(d.C);
    d4 cin[TM][TN];
    if (beta != 0.0) {
#pragma unroll
        for (int ti = 0; ti < TM; ++ti) {
            const int gi = i0 + ti * 16 + lr;
            const uint32_t gic = (uint32_t)(gi < m ? gi : m - 1);
#pragma unroll
            for (int tj = 0; tj < TN; ++tj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gj = j0 + tj * 16 + lg + 4 * r;
                    const uint32_t gjc = (uint32_t)(gj < n ? gj : n - 1);
                    cin[ti][tj][r] = at(C, (gic + gjc * ldc) * 8u);
                }
        }
    }

    d4 acc[TM][TN];
#pragma unroll
    for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TN; ++tj)
            acc[ti][tj] = d4{0.0, 0.0, 0.0, 0.0};

    const int kfull = K & ~15;
    const double *Ak = uni(d.A), *Bk = uni(d.B);  // wave-uniform chunk bases
    auto load_chunk = [&](double (&xa)[TM][4], double (&xb)[TN][4]) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int ti = 0; ti < TM; ++ti)
                xa[ti][s] = at(Ak, (oa[ti] + (uint32_t)s * ska) * 8u);
#pragma unroll
            for (int tj = 0; tj < TN; ++tj)
                xb[tj][s] = at(Bk, (ob[tj] + (uint32_t)s * skb) * 8u);
        }
    };
    auto mfma_chunk = [&](const double (&xa)[TM][4], const double (&xb)[TN][4]) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                for (int tj = 0; tj < TN; ++tj)
                    acc[ti][tj] = mfma16(xb[tj][s], xa[ti][s], acc[ti][tj]);
    };

    double fa[TM][4], fb[TN][4];
    for (int kk = 0; kk < kfull; kk += 16) {
        load_chunk(fa, fb);
        Ak += 16 * (size_t)ska;
        Bk += 16 * (size_t)skb;
        mfma_chunk(fa, fb);
    }
    if (kfull < K) {
        // k tail: one chunk with k clamped to K - 1 and zeroed past K
        const uint32_t last = (uint32_t)(K - 1 - kfull);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const uint32_t k = (uint32_t)(4 * lg + s);
            const bool kok = k <= last;
            const uint32_t dk = (kok ? k : last) - (uint32_t)(4 * lg);  // may wrap: offsets are modular
#pragma unroll
            for (int ti = 0; ti < TM; ++ti) {
                const double v = at(Ak, (oa[ti] + dk * ska) * 8u);
                fa[ti][s] = kok ? v : 0.0;
            }
#pragma unroll
            for (int tj = 0; tj < TN; ++tj) {
                const double v = at(Bk, (ob[tj] + dk * skb) * 8u);
                fb[tj][s] = kok ? v : 0.0;
            }
        }
        mfma_chunk(fa, fb);
    }
#pragma unroll
    for (int ti = 0; ti < TM; ++ti) {
        const int gi = i0 + ti * 16 + lr;
#pragma unroll
        for (int tj = 0; tj < TN; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gj = j0 + tj * 16 + lg + 4 * r;
                if (gi < m && gj < n) {
                    const double v = acc[ti][tj][r];
                    at(C, ((uint32_t)gi + (uint32_t)gj * ldc) * 8u) =
                        (beta == 0.0) ? alpha * v : fma(alpha, v, beta * cin[ti][tj][r]);
                }
            }
    }
}

// Dispatch one dgemm unit on its kind (trans case and register tile).
__device__ __forceinline__ void gemm_unit(const FusedDesc &d, int kind, uint32_t tile, int lane)
{
#define MB_FUSED_CASE(KIND, TA, TB, TM, TN)          \
    case KIND:                                       \
        regtile<TA, TB, TM, TN>(d, tile, lane);      \
        break;
    switch (kind) {
        MB_FUSED_CASE(0, false, false, 1, 1)
        MB_FUSED_CASE(1, false, true, 1, 1)
        MB_FUSED_CASE(2, true, false, 1, 1)
        MB_FUSED_CASE(3, true, true, 1, 1)
        MB_FUSED_CASE(4, false, false, 2, 1)
        MB_FUSED_CASE(5, false, true, 2, 1)
        MB_FUSED_CASE(6, true, false, 2, 1)
        MB_FUSED_CASE(7, true, true, 2, 1)
        MB_FUSED_CASE(8, false, false, 1, 2)
        MB_FUSED_CASE(9, false, true, 1, 2)
        MB_FUSED_CASE(10, true, false, 1, 2)
        MB_FUSED_CASE(11, true, true, 1, 2)
        MB_FUSED_CASE(12, false, false, 2, 2)
        MB_FUSED_CASE(13, false, true, 2, 2)
        MB_FUSED_CASE(14, true, false, 2, 2)
        MB_FUSED_CASE(15, true, true, 2, 2)
    default:
        break;
    }
#undef MB_FUSED_CASE
}

constexpr int FUSED_WAVES = 4;  // waves per workgroup, each an independent worker

// Claim the next unit of a queue: one atomic per wave, issued by lane 0.
__device__ __forceinline__ int claim(int *ctr, int lane)
{
    int v = 0;
    if (lane == 0)
        v = atomicAdd(ctr, 1);
    return __builtin_amdgcn_readfirstlane(v);
}

__global__ __launch_bounds__(FUSED_WAVES * 64) void fused_kernel(FusedArgs p)
{
    __shared__ PotrfSmem smem[FUSED_WAVES];
    const int lane = threadIdx.x & 63;
    PotrfSmem &S = smem[threadIdx.x >> 6];
    const int home = (int)(blockIdx.x % FUSED_QUEUES);  // the XCD this workgroup runs on
    for (int qi = 0; qi < FUSED_QUEUES; ++qi) {
        const int q = (home + qi) % FUSED_QUEUES;
        const int beg = p.qoff[q], cnt = p.qoff[q + 1] - beg;
        int *ctr = p.counters + q * FUSED_CTR_STRIDE;
        for (int u = claim(ctr, lane); u < cnt; u = claim(ctr, lane)) {
            const FusedUnit w = p.units[beg + u];
            const FusedDesc &d = p.desc[uni(w.prob)];
            const int kind = uni(d.kind);
            if (kind == FUSED_POTRF) {
                const int n = uni(d.n);
                const int info =
                    potrf_wave<false>(uni(d.C), (size_t)uni(d.ldc), n, (n + 15) / 16, S, lane);
                if (lane == 0)
                    *global_ptr(d.info) = info;
            } else {
                gemm_unit(d, kind, uni(w.tile), lane);
            }
        }
    }
}

// Zero the queue counters (a kernel rather than a memset, so that the reset
// can sit in a captured graph).
__global__ void fused_reset_kernel(int *counters)
{
    const int q = threadIdx.x;
    if (q < FUSED_QUEUES)
        counters[q * FUSED_CTR_STRIDE] = 0;
}

// dst[i][0] = src[i]: per-problem info words from a contiguous batch result.
__global__ void scatter_info_kernel(const int *src, int *const *dst, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        *global_ptr(dst[i]) = src[i];
}

hipError_t fused_grid(int *grid, int *waves_per_cu)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fused_kernel, FUSED_WAVES * 64, 0);
    if (e != hipSuccess)
        return e;
    if (per_cu < 1)
        per_cu = 1;
    *grid = cus * per_cu;
    if (waves_per_cu)
        *waves_per_cu = per_cu * FUSED_WAVES;
    return hipSuccess;
}

hipError_t launch_fused(const FusedArgs &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(fused_reset_kernel, dim3(1), dim3(64), 0, s, a.counters);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(fused_kernel, dim3((unsigned)grid), dim3(FUSED_WAVES * 64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scatter_info(const int *src, int *const *dst, int count, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(scatter_info_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       src, dst, count);
    return hipGetLastError();
}

}  // namespace mb
