// potrf_adj.hip -- batched reverse-mode derivative of the lower Cholesky
// factorization (one wave per instance, potrf_adj_wave.h), and the batched
// dlaset used to clear the unreferenced triangle of a factor.
#include "potrf_adj_wave.h"

namespace mb {

constexpr int ADJ_IPB = 4;  // instances (waves) per workgroup

__global__ __launch_bounds__(ADJ_IPB * 64) void potrf_adj_kernel(PotrfAdjArgs p)
{
    __shared__ AdjSmem smem[ADJ_IPB];
    const int lane = threadIdx.x & 63;
    const int inst = threadIdx.x >> 6;
    const int64_t b = (int64_t)blockIdx.x * ADJ_IPB + inst;
    if (b >= p.batch)
        return;
    const double *L = inst_ptr(p.L, p.Larr, p.sL, b);
    const double *Lb = inst_ptr(p.Lbar, p.Lbararr, p.sLbar, b);
    double *Ab = inst_ptr(p.Abar, p.Abararr, p.sAbar, b);
    potrf_adj_wave(L, (size_t)p.ldl, Lb, (size_t)p.ldlb, Ab, (size_t)p.ldab, p.n, (p.n + 15) / 16,
                   smem[inst], lane);
}

// Orders up to 64: every tile in registers (potrf_adj_regs), one kernel per
// tile count.
template <int NT>
__global__ __launch_bounds__(ADJ_IPB * 64) void potrf_adj_regs_kernel(PotrfAdjArgs p)
{
    __shared__ AdjSmem smem[ADJ_IPB];
    const int lane = threadIdx.x & 63;
    const int inst = threadIdx.x >> 6;
    const int64_t b = (int64_t)blockIdx.x * ADJ_IPB + inst;
    if (b >= p.batch)
        return;
    const double *L = inst_ptr(p.L, p.Larr, p.sL, b);
    const double *Lb = inst_ptr(p.Lbar, p.Lbararr, p.sLbar, b);
    double *Ab = inst_ptr(p.Abar, p.Abararr, p.sAbar, b);
    potrf_adj_regs<NT>(L, (size_t)p.ldl, Lb, (size_t)p.ldlb, Ab, (size_t)p.ldab, p.n, smem[inst],
                       lane);
}

hipError_t launch_potrf_adj(const PotrfAdjArgs &a, hipStream_t s)
{
    const int64_t blocks = ((int64_t)a.batch + ADJ_IPB - 1) / ADJ_IPB;
    const dim3 grid((unsigned)blocks), block(64 * ADJ_IPB);
    switch ((a.n + 15) / 16) {
    case 1: hipLaunchKernelGGL(potrf_adj_regs_kernel<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(potrf_adj_regs_kernel<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(potrf_adj_regs_kernel<3>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(potrf_adj_regs_kernel<4>, grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL(potrf_adj_kernel, grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

// dlaset: the strictly upper (uplo 0), strictly lower (uplo 1) or all
// off-diagonal (uplo 2) elements of the m x n matrix become alpha, the
// diagonal beta.  One thread per element, grid (elements / 256, batch).
__global__ void laset_kernel(LasetArgs p)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = blockIdx.y + (int64_t)gridDim.y * blockIdx.z;
    if (b >= p.batch || e >= (int64_t)p.m * p.n)
        return;
    const int i = (int)(e % p.m), j = (int)(e / p.m);
    double *A = inst_ptr(p.A, p.Aarr, p.sA, b);
    const bool sel = (i == j) || (p.uplo == 0 ? i < j : (p.uplo == 1 ? i > j : true));
    if (sel)
        global_ptr(A)[(size_t)i + (size_t)j * (size_t)p.lda] = (i == j) ? p.beta : p.alpha;
}

hipError_t launch_laset(const LasetArgs &a, hipStream_t s)
{
    const int64_t elems = (int64_t)a.m * a.n;
    if (elems == 0 || a.batch == 0)
        return hipSuccess;
    const unsigned gx = (unsigned)((elems + 255) / 256);
    const unsigned gy = (unsigned)(a.batch < 65535 ? a.batch : 65535);
    const unsigned gz = (unsigned)((a.batch + gy - 1) / gy);
    hipLaunchKernelGGL(laset_kernel, dim3(gx, gy, gz), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace mb
