// trmm_syrk.hip -- batched dtrmm (side 'R', uplo 'L', trans 'N', diag 'N')
// and dsyrk (uplo 'L', trans 'N'): the two BLAS routines the Riccati
// recursion of Sec. 5.2 calls besides dpotrf, for callers that compose the
// recursion from library calls rather than using the fused kernel.
//
// dtrmm  B <= alpha * B * A  (B m x n, A n x n lower, in place): one wave per
//   16-row block of B.  The wave produces the block's column tiles K in
//   increasing order, tile K = sum_{T >= K} B(I,T) A(T,K) in 16 x 16 FP64
//   MFMA tiles (A's tiles read transposed, its strictly upper part masked), so
//   every tile of B is read before the wave overwrites it (Sec. 3.1.4: the
//   triangular operand on the right, like the right-variant dtrsm).
// dsyrk  lower triangle of C <= alpha * A * A^T + beta * C (C n x n, A n x k):
//   one wave per lower tile (I,J) of C, sum_K A(I,K) A(J,K)^T in MFMA tiles;
//   on diagonal tiles only the lower part is written (Sec. 3.1.2).
#include "mb_internal.h"

namespace mb {

constexpr int TS_WPB = 4;  // waves per workgroup, each an independent tile worker

__device__ __forceinline__ d4 ts_xyT(d4 acc, const d4 &x, const d4 &y)
{
#pragma unroll
    for (int s = 0; s < 4; ++s)
        acc = mfma16(y[s], x[s], acc);
    return acc;
}

// Tile (I, T) of the rows x cols matrix X (accumulator order), zero outside.
__device__ __forceinline__ d4 ts_load(const MB_GLOBAL double *X, size_t ld, int rows, int cols, int I,
                                      int T, int lr, int lg)
{
    d4 t;
    const int gi = 16 * I + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gc = 16 * T + lg + 4 * r;
        t[r] = (gi < rows && gc < cols) ? X[(size_t)gi + (size_t)gc * ld] : 0.0;
    }
    return t;
}

// Transpose of tile (T, K) of the n x n lower triangle of A.
__device__ __forceinline__ d4 ts_load_lower_t(const MB_GLOBAL double *A, size_t ld, int n, int T, int K,
                                              int lr, int lg)
{
    d4 t;
    const int col = 16 * K + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * T + lg + 4 * r;
        t[r] = (row < n && col < n && row >= col) ? A[(size_t)row + (size_t)col * ld] : 0.0;
    }
    return t;
}

__global__ __launch_bounds__(TS_WPB * 64) void trmm_rlnn_kernel(TrmmArgs p, int tiles_m, int64_t w0)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = w0 + (int64_t)blockIdx.x * TS_WPB + (threadIdx.x >> 6);
    if (wid >= (int64_t)tiles_m * p.batch)
        return;
    const int64_t b = wid / tiles_m;
    const int I = (int)(wid - b * tiles_m);
    const int lr = lane & 15, lg = lane >> 4;
    const MB_GLOBAL double *A = global_ptr(p.A) + b * p.sA;
    MB_GLOBAL double *B = global_ptr(p.B) + b * p.sB;
    const int nt = (p.n + 15) / 16;
    for (int K = 0; K < nt; ++K) {
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
        if (p.alpha != 0.0)
            for (int T = K; T < nt; ++T)
                acc = ts_xyT(acc, ts_load(B, (size_t)p.ldb, p.m, p.n, I, T, lr, lg),
                             ts_load_lower_t(A, (size_t)p.lda, p.n, T, K, lr, lg));
        const int gi = 16 * I + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gc = 16 * K + lg + 4 * r;
            if (gi < p.m && gc < p.n)
                B[(size_t)gi + (size_t)gc * p.ldb] = p.alpha * acc[r];
        }
    }
}

__global__ __launch_bounds__(TS_WPB * 64) void syrk_ln_kernel(SyrkArgs p, int tiles, int64_t w0)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = w0 + (int64_t)blockIdx.x * TS_WPB + (threadIdx.x >> 6);
    if (wid >= (int64_t)tiles * p.batch)
        return;
    const int64_t b = wid / tiles;
    int t = (int)(wid - b * tiles);
    // lower tile t -> (I, J), J <= I, row by row
    int I = 0;
    while (t > I) {
        t -= I + 1;
        ++I;
    }
    const int J = t;
    const int lr = lane & 15, lg = lane >> 4;
    const MB_GLOBAL double *A = global_ptr(p.A) + b * p.sA;
    MB_GLOBAL double *C = global_ptr(p.C) + b * p.sC;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    if (p.alpha != 0.0)
        for (int K = 0; K < (p.k + 15) / 16; ++K)
            acc = ts_xyT(acc, ts_load(A, (size_t)p.lda, p.n, p.k, I, K, lr, lg),
                         ts_load(A, (size_t)p.lda, p.n, p.k, J, K, lr, lg));
    const int gi = 16 * I + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gc = 16 * J + lg + 4 * r;
        if (gi < p.n && gc <= gi) {
            MB_GLOBAL double *c = C + (size_t)gi + (size_t)gc * p.ldc;
            *c = p.beta == 0.0 ? p.alpha * acc[r] : p.alpha * acc[r] + p.beta * *c;
        }
    }
}

// Launch `waves` tile workers in slices of at most 2^30 workgroups.
template <class Args>
static hipError_t ts_launch(void (*kern)(Args, int, int64_t), const Args &a, int tiles,
                            int64_t waves, hipStream_t s)
{
    constexpr int64_t slice = ((int64_t)1 << 30) * TS_WPB;
    for (int64_t w0 = 0; w0 < waves; w0 += slice) {
        const int64_t n = std::min(slice, waves - w0);
        hipLaunchKernelGGL(kern, dim3((unsigned)((n + TS_WPB - 1) / TS_WPB)), dim3(TS_WPB * 64), 0,
                           s, a, tiles, w0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_trmm_rlnn(const TrmmArgs &a, hipStream_t s)
{
    const int tiles_m = (a.m + 15) / 16;
    return ts_launch(trmm_rlnn_kernel, a, tiles_m, (int64_t)tiles_m * a.batch, s);
}

hipError_t launch_syrk_ln(const SyrkArgs &a, hipStream_t s)
{
    const int nt = (a.n + 15) / 16;
    const int tiles = nt * (nt + 1) / 2;
    return ts_launch(syrk_ln_kernel, a, tiles, (int64_t)tiles * a.batch, s);
}

}  // namespace mb
