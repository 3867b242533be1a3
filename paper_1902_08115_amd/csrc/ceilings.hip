// ceilings.hip -- measured compute ceilings of the device (roofline support).
//
// Register-only loops whose flop count is known exactly: back-to-back FP64
// matrix-core steps (v_mfma_f64_16x16x4, 2048 flop per wave and step) and
// FP64 vector FMAs (2 flop per lane).  Each wave keeps several independent
// accumulator chains so that the pipes stay busy; the results are stored
// once so that nothing is optimised away.  Timed by the caller, they give the
// sustained FP64 peaks at the clock the device holds under such load -- the
// figures the achieved rates of the kernels can be read against next to the
// vendor's specification.
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

}  // namespace mb

extern "C" {

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
