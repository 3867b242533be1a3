// fused.hip -- one persistent kernel for an uneven batch of dgemm and dpotrf
// problems of mixed sizes.
//
// The paper switches between kernel variants by operand size (Sec. 2.4) but
// leaves batching aside; a batch whose problems all differ in shape cannot be
// served by per-shape launches without paying one launch per shape.  Here a
// plan (plan.hip) turns the batch into tasks -- one register tile of a dgemm,
// or one whole dpotrf -- sorted by estimated cost and dealt to one queue per
// XCD.  Every wave of the persistent grid is an independent worker: it claims
// the next task of its XCD's queue with one atomic increment, runs it, and
// moves on to the other queues once its own is empty, so the grid drains every
// queue whatever the dispatch order.
//
// The work is latency-bound per wave, so the loop keeps memory requests in
// flight at every step: the index of the task after next is claimed, and the
// next task is fetched (scalar loads, it is wave-uniform), while the current
// one runs; inside a dgemm tile the operands of k chunk c + 1 are loaded
// while the matrix cores work on chunk c.
//
// dgemm tasks are TM x TN tiles of 16 x 16 FP64 MFMA blocks computed straight
// from global memory: within one wave the operand fragments of a 16-deep k
// chunk partition the A and B panels exactly (lane (g, i) holds k = kk + 4g +
// s, s = 0..3, of row i), so there is no redundant load to share through LDS
// and no LDS traffic or barrier at all.  As in the batched kernels the MFMA
// takes op(B) as its left operand and accumulates C^T, so a lane owns whole
// rows of C and the epilogue stores are coalesced along columns.  dpotrf tasks
// run the batched kernel's per-wave factorization.
#include "potrf_wave.h"

namespace mb {

__device__ __forceinline__ MB_GLOBAL double &at(double *base, uint32_t byte_off)
{
    return *(MB_GLOBAL double *)((MB_GLOBAL char *)global_ptr(base) + byte_off);
}
__device__ __forceinline__ const MB_GLOBAL double &at(const double *base, uint32_t byte_off)
{
    return *(const MB_GLOBAL double *)((const MB_GLOBAL char *)global_ptr(base) + byte_off);
}

// Four consecutive doubles at base + byte_off as two 16-byte loads (the
// address is only known to be 8-byte aligned, which the 16-byte global load
// form accepts).
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
__device__ __forceinline__ void load4(const double *base, uint32_t byte_off, double (&x)[4])
{
    const MB_GLOBAL d2u *p =
        (const MB_GLOBAL d2u *)((const MB_GLOBAL char *)global_ptr(base) + byte_off);
    const d2u v0 = p[0], v1 = p[1];
    x[0] = v0.x;
    x[1] = v0.y;
    x[2] = v1.x;
    x[3] = v1.y;
}

// One register tile: C(i0:i0+16TM, j0:j0+16TN) <= alpha op(A) op(B) + beta C.
//
// op(A)[i][k] lives at A[i + k lda] ('N') or A[k + i lda] ('T'); op(B)[k][j]
// at B[k + j ldb] ('N') or B[j + k ldb] ('T').  Rows of op(A) past m and
// columns of op(B) past n read a clamped in-range address instead: entry
// (i, j) of the product depends on row i of op(A) and column j of op(B) only,
// so the padded lanes affect just the C entries that are never stored.  Slots
// past K read in-range addresses and are zeroed, since every output sums over
// k.  No load is ever predicated off, so the chunk loop has no branch and the
// loads of chunk c + 1 stay in flight across the MFMAs of chunk c.
//
// Addresses are a wave-uniform base plus a 32-bit byte offset per lane (the
// scalar-base + vector-offset form of the global loads); plans check that
// every operand spans less than 4 GiB.
template <bool TA, bool TB, int TM, int TN>
__device__ __forceinline__ void regtile(const FusedTask &t, int lane)
{
    const int lr = lane & 15, lg = lane >> 4;
    const int i0 = t.i0, j0 = t.j0;
    const int m = t.m, n = t.n, K = t.k;
    const uint32_t lda = (uint32_t)t.lda, ldb = (uint32_t)t.ldb, ldc = (uint32_t)t.ldc;
    const uint32_t ska = TA ? 1u : lda;  // element step along k in A
    const uint32_t skb = TB ? ldb : 1u;  // element step along k in B
    const double *A = t.A, *B = t.B;
    double *C = t.C;

    // per-lane element offset of k = 0 in each fragment row / column
    uint32_t ra[TM], rb[TN];
#pragma unroll
    for (int ti = 0; ti < TM; ++ti) {
        const int i = i0 + ti * 16 + lr;
        const uint32_t ic = (uint32_t)(i < m ? i : m - 1);
        ra[ti] = TA ? ic * lda : ic;
    }
#pragma unroll
    for (int tj = 0; tj < TN; ++tj) {
        const int j = j0 + tj * 16 + lr;
        const uint32_t jc = (uint32_t)(j < n ? j : n - 1);
        rb[tj] = TB ? jc : jc * ldb;
    }

    const double alpha = t.alpha, beta = t.beta;
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

    // Chunk c covers k = 16c + 4 lg + s, s = 0..3, for lane group lg.  The
    // four k of a lane are consecutive, so an operand stored along k ('T' A,
    // 'N' B) is read with two 16-byte loads per fragment.  In the last chunk
    // a group that crosses K starts at K - 4 instead (the order of k inside
    // a chunk is free as long as A and B agree): its first slots then repeat
    // k of the previous group and are zeroed, as are groups past K, and no
    // address ever passes K - 1.  Needs K >= 4; smaller K take the clamped
    // single-chunk path below.
    auto group_start = [&](int c) {
        const int kb = 16 * c + 4 * lg;
        return kb < K - 4 ? kb : K - 4;
    };
    auto load_chunk = [&](int c, double (&xa)[TM][4], double (&xb)[TN][4]) {
        const uint32_t kg = (uint32_t)group_start(c);
#pragma unroll
        for (int ti = 0; ti < TM; ++ti) {
            if constexpr (TA) {
                load4(A, (ra[ti] + kg) * 8u, xa[ti]);
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    xa[ti][s] = at(A, (ra[ti] + (kg + (uint32_t)s) * lda) * 8u);
            }
        }
#pragma unroll
        for (int tj = 0; tj < TN; ++tj) {
            if constexpr (!TB) {
                load4(B, (rb[tj] + kg) * 8u, xb[tj]);
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    xb[tj][s] = at(B, (rb[tj] + (kg + (uint32_t)s) * ldb) * 8u);
            }
        }
    };
    auto mfma_chunk = [&](int c, const double (&xa)[TM][4], const double (&xb)[TN][4]) {
        const int kb = 16 * c + 4 * lg;
        const int kg = group_start(c);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bool keep = kg + s >= kb;
#pragma unroll
            for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                for (int tj = 0; tj < TN; ++tj)
                    acc[ti][tj] = mfma16(keep ? xb[tj][s] : 0.0, keep ? xa[ti][s] : 0.0,
                                         acc[ti][tj]);
        }
    };

    const int nch = (K + 15) >> 4;
    if (K >= 4) {
        double fa[TM][4], fb[TN][4];
        load_chunk(0, fa, fb);
        for (int c = 0; c < nch; ++c) {
            double ga[TM][4], gb[TN][4];
            load_chunk(c + 1 < nch ? c + 1 : c, ga, gb);  // the last one re-reads (cache hits)
            mfma_chunk(c, fa, fb);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
#pragma unroll
                for (int ti = 0; ti < TM; ++ti)
                    fa[ti][s] = ga[ti][s];
#pragma unroll
                for (int tj = 0; tj < TN; ++tj)
                    fb[tj][s] = gb[tj][s];
            }
        }
    } else if (K > 0) {
        // 1 <= K <= 3: one chunk, lane group 0 only, k clamped and zeroed past K
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bool keep = lg == 0 && s < K;
            const uint32_t k = (uint32_t)(s < K ? s : K - 1);
            double xa[TM], xb[TN];
#pragma unroll
            for (int ti = 0; ti < TM; ++ti)
                xa[ti] = at(A, (ra[ti] + k * ska) * 8u);
#pragma unroll
            for (int tj = 0; tj < TN; ++tj)
                xb[tj] = at(B, (rb[tj] + k * skb) * 8u);
#pragma unroll
            for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                for (int tj = 0; tj < TN; ++tj)
                    acc[ti][tj] = mfma16(keep ? xb[tj] : 0.0, keep ? xa[ti] : 0.0, acc[ti][tj]);
        }
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

// Run one task (kind is wave-uniform).
__device__ __forceinline__ void run_task(const FusedTask &t, PotrfSmem &S, int lane)
{
#define MB_FUSED_CASE(KIND, TA, TB, TM, TN) \
    case KIND:                              \
        regtile<TA, TB, TM, TN>(t, lane);   \
        break;
    switch (t.kind) {
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
#ifndef FUSED_NO_POTRF
    case FUSED_POTRF: {
        const int info = potrf_wave<true>(t.C, (size_t)t.ldc, t.n, (t.n + 15) / 16, S, lane);
        if (lane == 0)
            *global_ptr(t.info) = info;
        break;
    }
#endif
    default:
        break;
    }
#undef MB_FUSED_CASE
}

constexpr int FUSED_WAVES = 4;  // waves per workgroup, each an independent worker

// Claim the next task of a queue: one atomic per wave, issued by lane 0.  The
// result stays in lane 0's register until claim_get reads it, so the atomic's
// latency overlaps whatever the wave does in between.
__device__ __forceinline__ int claim_issue(int *ctr, int lane)
{
    int v = 0;
    if (lane == 0)
        v = atomicAdd(ctr, 1);
    return v;
}
__device__ __forceinline__ int claim_get(int v) { return __builtin_amdgcn_readfirstlane(v); }

// The restrict-qualified read-only task table lets the compiler fetch tasks
// with scalar loads straight into scalar registers.
__global__ __launch_bounds__(FUSED_WAVES * 64) void fused_kernel(
    const FusedTask *__restrict__ tasks, const int *__restrict__ qoff, int *counters)
{
    __shared__ PotrfSmem smem[FUSED_WAVES];
    const int lane = threadIdx.x & 63;
    PotrfSmem &S = smem[threadIdx.x >> 6];
    const int home = (int)(blockIdx.x % FUSED_QUEUES);  // the XCD this workgroup runs on
    for (int qi = 0; qi < FUSED_QUEUES; ++qi) {
        const int q = (home + qi) % FUSED_QUEUES;
        const int beg = qoff[q], cnt = qoff[q + 1] - beg;
        int *ctr = counters + q * FUSED_CTR_STRIDE;
        int u = claim_get(claim_issue(ctr, lane));
        if (u >= cnt)
            continue;
        FusedTask cur = tasks[beg + u];
        u = claim_get(claim_issue(ctr, lane));
        for (;;) {
            // fetch the next task and claim the one after it; both complete
            // while the current task runs
            const bool more = u < cnt;
            FusedTask nxt;
            int raw = 0;
            if (more) {
                nxt = tasks[beg + u];
                raw = claim_issue(ctr, lane);
            }
            run_task(cur, S, lane);
            if (!more)
                break;
            cur = nxt;
            u = claim_get(raw);
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
    hipLaunchKernelGGL(fused_kernel, dim3((unsigned)grid), dim3(FUSED_WAVES * 64), 0, s, a.tasks,
                       a.qoff, a.counters);
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
