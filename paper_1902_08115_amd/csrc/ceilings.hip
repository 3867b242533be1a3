// ceilings.hip -- measured ceilings of the device (roofline support).
//
// Register-only loops whose flop count is known exactly: back-to-back FP64
// matrix-core steps (v_mfma_f64_16x16x4, 2048 flop per wave and step) and
// FP64 vector FMAs (2 flop per lane).  Each wave keeps several independent
// accumulator chains so that the pipes stay busy; the results are stored
// once so that nothing is optimised away.  Timed by the caller, they give the
// sustained FP64 peaks at the clock the device holds under such load -- the
// figures the achieved rates of the kernels can be read against next to the
// vendor's specification.
//
// The HBM probes stream a buffer far larger than every cache level with
// 16-byte loads and stores, four of them in flight per thread before the
// first is used: read only (a per-thread sum is stored), copy, and three
// reads per write (the read:write mix of a dgemm with beta != 0).
#include "mi355blas.h"
#include "mb_internal.h"

namespace mb {

constexpr int CEIL_THREADS = 256;

__global__ __launch_bounds__(CEIL_THREADS) void ceiling_mfma_kernel(int iters, double seed,
                                                                    double *out)
{
    const int lane = threadIdx.x & 63;
    const double a = seed + 1e-3 * lane, b = seed - 1e-3 * lane;
    d4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
        acc[c] = d4{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            acc[c] = mfma16(a, b, acc[c]);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c)
        s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[(size_t)blockIdx.x * CEIL_THREADS + threadIdx.x] = s;
}

__global__ __launch_bounds__(CEIL_THREADS) void ceiling_fma_kernel(int iters, double seed,
                                                                   double *out)
{
    const double a = 1.0 - 1e-9, b = seed * 1e-9;
    double x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c)
        x[c] = seed + c + threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
            x[c] = fma(x[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c)
        s += x[c];
    out[(size_t)blockIdx.x * CEIL_THREADS + threadIdx.x] = s;
}

// HBM streaming probes over 16-byte elements (pairs of doubles).  Each
// thread handles U consecutive grid strides per round so that U independent
// loads are in flight; the remainder past the last whole round is taken one
// element at a time.  kind 0: read src[0, n2); kind 1: dst = src; kind 2:
// dst = src0 + src1 + src2 with src_j = src + j * n2.
typedef double d2 __attribute__((ext_vector_type(2)));

template <int KIND>
__global__ __launch_bounds__(CEIL_THREADS) void ceiling_hbm_kernel(const d2 *__restrict__ src,
                                                                   d2 *__restrict__ dst,
                                                                   int64_t n2, double *out)
{
    constexpr int U = 4;
    const int64_t stride = (int64_t)gridDim.x * CEIL_THREADS;
    const int64_t tid = (int64_t)blockIdx.x * CEIL_THREADS + threadIdx.x;
    d2 acc = d2{0.0, 0.0};
    const int64_t whole = n2 / (stride * U) * (stride * U);
    for (int64_t base = tid; base < whole; base += stride * U) {
        d2 v[U];
        if (KIND == 2) {
            d2 w[U], x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                v[u] = __builtin_nontemporal_load(src + base + u * stride);
                w[u] = __builtin_nontemporal_load(src + n2 + base + u * stride);
                x[u] = __builtin_nontemporal_load(src + 2 * n2 + base + u * stride);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                __builtin_nontemporal_store(v[u] + w[u] + x[u], dst + base + u * stride);
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
                v[u] = __builtin_nontemporal_load(src + base + u * stride);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (KIND == 0)
                    acc += v[u];
                else
                    __builtin_nontemporal_store(v[u], dst + base + u * stride);
            }
        }
    }
    for (int64_t i = whole + tid; i < n2; i += stride) {
        if (KIND == 0)
            acc += src[i];
        else if (KIND == 1)
            dst[i] = src[i];
        else
            dst[i] = src[i] + src[n2 + i] + src[2 * n2 + i];
    }
    if (KIND == 0)
        out[tid] = acc[0] + acc[1];
}

}  // namespace mb

extern "C" {

int mb_ceiling_hbm(int kind, const double *src, double *dst, int64_t n, int blocks, double *out,
                   double *bytes, hipStream_t stream)
{
    if (kind < 0 || kind > 2)
        return -1;
    if (!src)
        return -2;
    if (kind != 0 && !dst)
        return -3;
    if (n <= 0 || (n & 1))
        return -4;
    if (blocks <= 0)
        return -5;
    if (kind == 0 && !out)
        return -6;
    if (!bytes)
        return -7;
    const int64_t n2 = n / 2;
    const mb::d2 *s2 = (const mb::d2 *)src;
    mb::d2 *t2 = (mb::d2 *)dst;
    const dim3 g((unsigned)blocks), b(mb::CEIL_THREADS);
    if (kind == 0) {
        hipLaunchKernelGGL(mb::ceiling_hbm_kernel<0>, g, b, 0, stream, s2, t2, n2, out);
        *bytes = 8.0 * (double)n;
    } else if (kind == 1) {
        hipLaunchKernelGGL(mb::ceiling_hbm_kernel<1>, g, b, 0, stream, s2, t2, n2, out);
        *bytes = 16.0 * (double)n;
    } else {
        hipLaunchKernelGGL(mb::ceiling_hbm_kernel<2>, g, b, 0, stream, s2, t2, n2, out);
        *bytes = 32.0 * (double)n;
    }
    return hipGetLastError() == hipSuccess ? MB_OK : MB_ERR_HIP;
}

int mb_ceiling_fp64(int kind, int blocks, int iters, double *out, double *flops,
                    hipStream_t stream)
{
    if (kind != 0 && kind != 1)
        return -1;
    if (blocks <= 0)
        return -2;
    if (iters <= 0)
        return -3;
    if (!out)
        return -4;
    if (!flops)
        return -5;
    if (kind == 0) {
        hipLaunchKernelGGL(mb::ceiling_mfma_kernel, dim3((unsigned)blocks), dim3(mb::CEIL_THREADS),
                           0, stream, iters, 1.0, out);
        *flops = (double)blocks * (mb::CEIL_THREADS / 64) * (double)iters * 4.0 * 2048.0;
    } else {
        hipLaunchKernelGGL(mb::ceiling_fma_kernel, dim3((unsigned)blocks), dim3(mb::CEIL_THREADS),
                           0, stream, iters, 1.0, out);
        *flops = (double)blocks * mb::CEIL_THREADS * (double)iters * 8.0 * 2.0;
    }
    return hipGetLastError() == hipSuccess ? MB_OK : MB_ERR_HIP;
}

}  // extern "C"
