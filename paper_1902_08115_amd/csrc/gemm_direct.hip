// gemm_direct.hip -- "direct" batched dgemm for tiny operands.
//
// The analogue of the paper's algorithmic variant 'D' (Sec. 2.2, Table 1):
// every operand is used in place, in its column-major layout, with no packing
// buffer.  On gfx950 that means operands go straight from global memory (L1/L2)
// into registers, with no LDS staging and no barriers.  One thread computes
// RN consecutive entries of one row of C; the threads of a 256-wide workgroup
// cover several whole instances (tiny m*n) or one slice of an instance.
// Consecutive lanes own consecutive rows i, so C and a non-transposed A are
// accessed with unit stride across lanes; op(B) values are shared by all lanes
// of an instance (broadcast loads).  At these sizes a thread's few products
// are cheap and its time is memory latency: the k loop goes in chunks of KC
// whose loads are all issued before the first product of the chunk, and C is
// read up front, so k <= KC costs one round trip instead of one per k step.
// KC = 4 measured best at every square size up to 16 (chunks of 8 hold more
// loads in flight but cost a wave per SIMD).  Whole chunks and the ragged
// last one are separate code: in a whole chunk a thread's k steps of one
// operand row or column, and (n a multiple of RN) its RN columns of a
// transposed B, are consecutive addresses that the compiler fetches with
// 16-byte loads -- fewer load instructions, which bound the rate at n = 8.
#include "mb_internal.h"

namespace mb {

// One chunk of KC k steps: all loads first, then the products in k order.
// FULL: every k step of the chunk exists; otherwise steps past the end load
// the last valid one and skip its product.
template <bool TA, bool TB, int RN, int KC, bool FULL>
__device__ __forceinline__ void direct_chunk(const double *A, const double *B, size_t lda,
                                             size_t ldb, int i, const int (&jc)[RN], int q0,
                                             int k, double (&acc)[RN])
{
    double av[KC], bv[KC][RN];
#pragma unroll
    for (int u = 0; u < KC; ++u) {
        const size_t q = (size_t)(FULL ? q0 + u : min(q0 + u, k - 1));
        av[u] = TA ? A[q + (size_t)i * lda] : A[(size_t)i + q * lda];
#pragma unroll
        for (int r = 0; r < RN; ++r)
            bv[u][r] = TB ? B[(size_t)jc[r] + q * ldb] : B[q + (size_t)jc[r] * ldb];
    }
#pragma unroll
    for (int u = 0; u < KC; ++u) {
        if (FULL || q0 + u < k) {
#pragma unroll
            for (int r = 0; r < RN; ++r)
                acc[r] = fma(av[u], bv[u][r], acc[r]);
        }
    }
}

// NC: n is a multiple of RN, so a thread's columns j0 .. j0 + RN - 1 all exist.
template <bool TA, bool TB, int RN, int KC, bool NC>
__global__ __launch_bounds__(256) void gemm_direct_kernel(GemmArgs p, int per_inst, int ipb)
{
    const int t = threadIdx.x;
    int64_t b;
    int rem;
    if (ipb > 0) {  // several instances per workgroup
        const int bl = t / per_inst;
        if (bl >= ipb)
            return;
        b = (int64_t)blockIdx.x * ipb + bl;
        rem = t - bl * per_inst;
    } else {  // one instance per blockIdx.x, its threads spread over blockIdx.y
        b = blockIdx.x;
        rem = (int)blockIdx.y * 256 + t;
        if (rem >= per_inst)
            return;
    }
    if (b >= p.batch)
        return;
    const int i = rem % p.m;
    const int j0 = (rem / p.m) * RN;

    const double *A = inst_ptr(p.A, p.Aarr, p.sA, b);
    const double *B = inst_ptr(p.B, p.Barr, p.sB, b);
    double *C = inst_ptr(p.C, p.Carr, p.sC, b);
    const size_t lda = (size_t)p.lda, ldb = (size_t)p.ldb, ldc = (size_t)p.ldc;
    const int k = p.k;  // >= 1 here: k == 0 never reaches this kernel

    // columns beyond n are clamped (read a valid column, result discarded)
    int jc[RN];
#pragma unroll
    for (int r = 0; r < RN; ++r)
        jc[r] = NC ? j0 + r : min(j0 + r, p.n - 1);

    // beta == 0: C is not read
    const bool read_c = p.beta != 0.0;
    double cv[RN];
#pragma unroll
    for (int r = 0; r < RN; ++r)
        cv[r] = read_c ? C[(size_t)i + (size_t)jc[r] * ldc] : 0.0;

    double acc[RN];
#pragma unroll
    for (int r = 0; r < RN; ++r)
        acc[r] = 0.0;

    // whole chunks, then the ragged last one: the sum runs over q = 0..k-1
    // in order either way
    int q0 = 0;
    for (; q0 + KC <= k; q0 += KC)
        direct_chunk<TA, TB, RN, KC, true>(A, B, lda, ldb, i, jc, q0, k, acc);
    if (q0 < k)
        direct_chunk<TA, TB, RN, KC, false>(A, B, lda, ldb, i, jc, q0, k, acc);
#pragma unroll
    for (int r = 0; r < RN; ++r) {
        const int j = j0 + r;
        if (NC || j < p.n)
            C[(size_t)i + (size_t)j * ldc] = read_c ? fma(p.alpha, acc[r], p.beta * cv[r])
                                                    : p.alpha * acc[r];
    }
}

// C <= beta*C (alpha == 0 or k == 0); beta == 0 writes zeros without reading C.
__global__ __launch_bounds__(256) void gemm_scale_kernel(GemmArgs p)
{
    const int64_t b = blockIdx.y;
    double *C = inst_ptr(p.C, p.Carr, p.sC, b);
    const int64_t mn = (int64_t)p.m * p.n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < mn; e += (int64_t)gridDim.x * 256) {
        const int j = (int)(e / p.m), i = (int)(e - (int64_t)j * p.m);
        double *c = C + (size_t)i + (size_t)j * (size_t)p.ldc;
        *c = (p.beta == 0.0) ? 0.0 : p.beta * (*c);
    }
}

template <bool TA, bool TB, bool NC>
static hipError_t launch_direct_n(const GemmArgs &a, hipStream_t s)
{
    constexpr int RN = 4, KC = 4;
    const int nb = (a.n + RN - 1) / RN;
    const int64_t per_inst64 = (int64_t)a.m * nb;
    if (per_inst64 > (int64_t)256 * 65535)
        return hipErrorInvalidValue;
    const int per_inst = (int)per_inst64;
    if (per_inst <= 256) {
        const int ipb = 256 / per_inst;
        const int64_t blocks = ((int64_t)a.batch + ipb - 1) / ipb;
        hipLaunchKernelGGL((gemm_direct_kernel<TA, TB, RN, KC, NC>), dim3((unsigned)blocks), dim3(256), 0,
                           s, a, per_inst, ipb);
    } else {
        const int gy = (per_inst + 255) / 256;
        hipLaunchKernelGGL((gemm_direct_kernel<TA, TB, RN, KC, NC>), dim3((unsigned)a.batch, gy),
                           dim3(256), 0, s, a, per_inst, 0);
    }
    return hipGetLastError();
}

template <bool TA, bool TB>
static hipError_t launch_direct_t(const GemmArgs &a, hipStream_t s)
{
    return a.n % 4 == 0 ? launch_direct_n<TA, TB, true>(a, s) : launch_direct_n<TA, TB, false>(a, s);
}

hipError_t launch_gemm_direct(bool ta, bool tb, const GemmArgs &a, hipStream_t s)
{
    if (!ta && !tb)
        return launch_direct_t<false, false>(a, s);
    if (!ta && tb)
        return launch_direct_t<false, true>(a, s);
    if (ta && !tb)
        return launch_direct_t<true, false>(a, s);
    return launch_direct_t<true, true>(a, s);
}

hipError_t launch_gemm_scale(const GemmArgs &a, hipStream_t s)
{
    const int64_t mn = (int64_t)a.m * a.n;
    int64_t gx = (mn + 255) / 256;
    if (gx > 1024)
        gx = 1024;
    int64_t done = 0;
    // grid.y is limited to 65535: split very large batches into several launches
    while (done < a.batch) {
        const int chunk = (int)((a.batch - done) > 65535 ? 65535 : (a.batch - done));
        GemmArgs sub = a;
        sub.batch = chunk;
        if (sub.Carr)
            sub.Carr = a.Carr + done;
        else
            sub.C = a.C + done * a.sC;
        hipLaunchKernelGGL(gemm_scale_kernel, dim3((unsigned)gx, chunk), dim3(256), 0, s, sub);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        done += chunk;
    }
    return hipSuccess;
}

}  // namespace mb
