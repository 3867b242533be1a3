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
// next task is fetched, while the current one runs; inside a dgemm tile the operands of k chunk c + 1 are loaded
// while the matrix cores work on chunk c.
//
// dgemm tasks are TM x TN tiles of 16 x 16 FP64 MFMA blocks computed straight
// from global memory: within one wave the operand fragments of a 16-deep k
// chunk partition the A and B panels exactly (lane (g, i) holds four k of row
// i, the four lane groups together all 16), so there is no redundant load to share through LDS
// and no LDS traffic or barrier at all.  As in the batched kernels the MFMA
// takes op(B) as its left operand and accumulates C^T, so a lane owns whole
// rows of C and the epilogue stores are coalesced along columns.  dpotrf and
// Cholesky-adjoint tasks run the batched kernels' per-wave routines.
#include "potrf_adj_wave.h"
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

// Two consecutive doubles at base + byte_off with one 16-byte load (the
// address is only known to be 8-byte aligned, which the 16-byte global load
// form accepts).
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
__device__ __forceinline__ void load2(const double *base, uint32_t byte_off, double &x0,
                                      double &x1)
{
    const d2u v = *(const MB_GLOBAL d2u *)((const MB_GLOBAL char *)global_ptr(base) + byte_off);
    x0 = v.x;
    x1 = v.y;
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

    // k runs in chunks of 16 with the remainder first: the head chunk covers
    // k < r = K - 16 (nch - 1), 1 <= r <= 16, and chunk c >= 1 covers
    // [r + 16 (c - 1), r + 16 c), always full.  In a chunk starting at k0,
    // slot s of lane group lg holds k = k0 + 8 (s/2) + 2 lg + (s%2): a lane's
    // slots are two pairs of consecutive k, and the four lane groups of one
    // row tile a contiguous 64-byte run per pair, so an operand stored along
    // k ('T' A, 'N' B) is read with one 16-byte load per pair, each load
    // instruction covering 64 contiguous bytes of every row it touches.  (The
    // order of k inside a chunk is free as long as A and B agree.)
    //
    // In the head, a pair that crosses r starts at r - 2 instead: its first
    // slot then repeats a k of the previous pair and is zeroed, as are pairs
    // past r, and no address passes r - 1; when r <= 8 the second pair is
    // skipped outright (a wave-uniform branch), and r == 1 uses slot 0 of lane
    // group 0 alone.  (The head's loads and MFMAs sit behind wave-uniform
    // branches, so the compiler waits for all loads before the head MFMAs;
    // from chunk 1 on, the loads of the next chunk overlap the MFMAs.)
    auto load_pair = [&](uint32_t ks, int p, double (&xa)[TM][4], double (&xb)[TN][4]) {
#pragma unroll
        for (int ti = 0; ti < TM; ++ti) {
            if constexpr (TA) {
                load2(A, (ra[ti] + ks) * 8u, xa[ti][2 * p], xa[ti][2 * p + 1]);
            } else {
                xa[ti][2 * p] = at(A, (ra[ti] + ks * lda) * 8u);
                xa[ti][2 * p + 1] = at(A, (ra[ti] + (ks + 1u) * lda) * 8u);
            }
        }
#pragma unroll
        for (int tj = 0; tj < TN; ++tj) {
            if constexpr (!TB) {
                load2(B, (rb[tj] + ks) * 8u, xb[tj][2 * p], xb[tj][2 * p + 1]);
            } else {
                xb[tj][2 * p] = at(B, (rb[tj] + ks * ldb) * 8u);
                xb[tj][2 * p + 1] = at(B, (rb[tj] + (ks + 1u) * ldb) * 8u);
            }
        }
    };
    auto mfma_slot = [&](int s, bool keep, const double (&xa)[TM][4], const double (&xb)[TN][4]) {
#pragma unroll
        for (int ti = 0; ti < TM; ++ti)
#pragma unroll
            for (int tj = 0; tj < TN; ++tj)
                acc[ti][tj] = mfma16(keep ? xb[tj][s] : 0.0, keep ? xa[ti][s] : 0.0, acc[ti][tj]);
    };
    auto load_full = [&](int c, double (&xa)[TM][4], double (&xb)[TN][4], int r) {
        const uint32_t k0 = (uint32_t)(r + 16 * (c - 1) + 2 * lg);
        load_pair(k0, 0, xa, xb);
        load_pair(k0 + 8u, 1, xa, xb);
    };
    auto mfma_full = [&](const double (&xa)[TM][4], const double (&xb)[TN][4]) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
            mfma_slot(s, true, xa, xb);
    };
    // head pair p: first k and whether slot e of it is new
    auto head_start = [&](int p, int r) {
        const int kn = 8 * p + 2 * lg;
        return kn < r - 2 ? kn : r - 2;
    };

    if (K == 1) {
        // one product term: slot 0 of lane group 0
        double fa[TM][4], fb[TN][4];
#pragma unroll
        for (int ti = 0; ti < TM; ++ti)
            fa[ti][0] = at(A, ra[ti] * 8u);
#pragma unroll
        for (int tj = 0; tj < TN; ++tj)
            fb[tj][0] = at(B, rb[tj] * 8u);
        mfma_slot(0, lg == 0, fa, fb);
    } else if (K >= 2) {
        const int nch = (K + 15) >> 4;
        const int r = K - 16 * (nch - 1);  // 2 <= r <= 16 unless K = 16 c + 1
        double fa[TM][4], fb[TN][4], ga[TM][4], gb[TN][4];
        if (r >= 2) {
            load_pair((uint32_t)head_start(0, r), 0, fa, fb);
            if (r > 8)
                load_pair((uint32_t)head_start(1, r), 1, fa, fb);
        } else {
#pragma unroll
            for (int ti = 0; ti < TM; ++ti)
                fa[ti][0] = at(A, ra[ti] * 8u);  // k = 0
#pragma unroll
            for (int tj = 0; tj < TN; ++tj)
                fb[tj][0] = at(B, rb[tj] * 8u);
        }
        if (nch > 1)
            load_full(1, ga, gb, r);  // in flight during the head's MFMAs
        if (r >= 2) {
#pragma unroll
            for (int s = 0; s < 2; ++s)
                mfma_slot(s, head_start(0, r) + s >= 2 * lg, fa, fb);
            if (r > 8) {
#pragma unroll
                for (int s = 2; s < 4; ++s)
                    mfma_slot(s, head_start(1, r) + (s & 1) >= 8 + 2 * lg, fa, fb);
            }
        } else {
            mfma_slot(0, lg == 0, fa, fb);  // k = 0 alone
        }
        if (nch > 1) {
            // chunk c + 1 is loaded before the MFMAs of chunk c
            for (int c = 2; c < nch; ++c) {
                double ha[TM][4], hb[TN][4];
                load_full(c, ha, hb, r);
                mfma_full(ga, gb);
#pragma unroll
                for (int s = 0; s < 4; ++s) {
#pragma unroll
                    for (int ti = 0; ti < TM; ++ti)
                        ga[ti][s] = ha[ti][s];
#pragma unroll
                    for (int tj = 0; tj < TN; ++tj)
                        gb[tj][s] = hb[tj][s];
                }
            }
            mfma_full(ga, gb);
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

// dlaset on columns [j0, j0 + FUSED_LASET_COLS) of the m x n matrix C; k is
// the part (0 strictly upper, 1 strictly lower, 2 all off-diagonal).
__device__ __forceinline__ void laset_task(const FusedTask &t, int lane)
{
    MB_GLOBAL double *C = global_ptr(t.C);
    const int j1 = min(t.j0 + FUSED_LASET_COLS, t.n);
    for (int j = t.j0; j < j1; ++j)
        for (int i = lane; i < t.m; i += 64) {
            const bool sel = i == j || (t.k == 0 ? i < j : (t.k == 1 ? i > j : true));
            if (sel)
                C[(size_t)i + (size_t)j * (size_t)t.ldc] = i == j ? t.beta : t.alpha;
        }
}

// Per-wave LDS of the dpotrf and Cholesky-adjoint tasks.
union TaskSmem {
    PotrfSmem potrf;
    AdjSmem adj;
};

// Run one task (kind is wave-uniform).
__device__ __forceinline__ void run_task(const FusedTask &t, TaskSmem &S, int lane)
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
    case FUSED_POTRF: {
        const int info =
            potrf_wave<true>(t.C, (size_t)t.ldc, t.n, (t.n + 15) / 16, S.potrf, lane);
        if (lane == 0)
            *global_ptr(t.info) = info;
        break;
    }
    case FUSED_POTRF_ADJ:
        potrf_adj_wave(t.A, (size_t)t.lda, t.B, (size_t)t.ldb, t.C, (size_t)t.ldc, t.n,
                       (t.n + 15) / 16, S.adj, lane);
        break;
    case FUSED_LASET:
        laset_task(t, lane);
        break;
    default:
        break;
    }
#undef MB_FUSED_CASE
}

constexpr int FUSED_WAVES = kFusedWaves;  // waves per workgroup, each an independent worker

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

// A task travels as one vector register: lane w < 24 holds dword w of the
// 96-byte record (one coalesced load), and the fields are read out with
// readlane when the task starts.  Two tasks in flight then cost two vector
// registers instead of 48 scalar ones.
__device__ __forceinline__ int task_fetch(const FusedTask *tasks, int idx, int lane)
{
    const MB_GLOBAL int *p = (const MB_GLOBAL int *)global_ptr(tasks + idx);
    return lane < 24 ? p[lane] : 0;
}
__device__ __forceinline__ uint32_t word(int v, int w)
{
    return (uint32_t)__builtin_amdgcn_readlane(v, w);
}
__device__ __forceinline__ uint64_t dword2(int v, int w)
{
    return (uint64_t)word(v, w) | ((uint64_t)word(v, w + 1) << 32);
}
__device__ __forceinline__ FusedTask task_unpack(int v)
{
    FusedTask t;
    t.A = (const double *)dword2(v, 0);
    t.B = (const double *)dword2(v, 2);
    t.C = (double *)dword2(v, 4);
    t.info = (int *)dword2(v, 6);
    t.alpha = __builtin_bit_cast(double, dword2(v, 8));
    t.beta = __builtin_bit_cast(double, dword2(v, 10));
    t.m = (int)word(v, 12);
    t.n = (int)word(v, 13);
    t.k = (int)word(v, 14);
    t.lda = (int)word(v, 15);
    t.ldb = (int)word(v, 16);
    t.ldc = (int)word(v, 17);
    t.kind = (int)word(v, 18);
    t.i0 = (int)word(v, 19);
    t.j0 = (int)word(v, 20);
    return t;
}

// Queue 2 x + c holds the class-c tasks (c = 0 dpotrf, 1 dgemm) meant for
// XCD x.  dpotrf tasks are long and latency-bound, dgemm tiles short and
// bandwidth-bound: the first potrf_waves waves of every workgroup start on
// the dpotrf class and the others on the dgemm class, so that both kinds run
// side by side instead of one phase after the other; a wave whose class is
// drained everywhere moves on to the other class.
__global__ __launch_bounds__(FUSED_WAVES * 64) void fused_kernel(const FusedTask *tasks,
                                                                 const int *qoff, int *counters,
                                                                 int potrf_waves)
{
    __shared__ TaskSmem smem[FUSED_WAVES];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    TaskSmem &S = smem[wave];
    const int home = (int)(blockIdx.x % FUSED_XCDS);  // the XCD this workgroup runs on
    const int first = wave < potrf_waves ? 0 : 1;
    for (int pass = 0; pass < FUSED_CLASSES; ++pass) {
        const int cls = pass == 0 ? first : 1 - first;
        for (int xi = 0; xi < FUSED_XCDS; ++xi) {
            const int q = FUSED_CLASSES * ((home + xi) % FUSED_XCDS) + cls;
            const int beg = qoff[q], cnt = qoff[q + 1] - beg;
            int *ctr = counters + q * FUSED_CTR_STRIDE;
            int u = claim_get(claim_issue(ctr, lane));
            if (u >= cnt)
                continue;
            int cur = task_fetch(tasks, beg + u, lane);
            u = claim_get(claim_issue(ctr, lane));
            for (;;) {
                // fetch the next task and claim the one after it; both
                // complete while the current task runs
                const bool more = u < cnt;
                int nxt = 0, raw = 0;
                if (more) {
                    nxt = task_fetch(tasks, beg + u, lane);
                    raw = claim_issue(ctr, lane);
                }
                run_task(task_unpack(cur), S, lane);
                if (!more)
                    break;
                cur = nxt;
                u = claim_get(raw);
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
    hipLaunchKernelGGL(fused_kernel, dim3((unsigned)grid), dim3(FUSED_WAVES * 64), 0, s, a.tasks,
                       a.qoff, a.counters, a.potrf_waves);
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
