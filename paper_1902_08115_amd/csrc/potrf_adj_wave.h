// potrf_adj_wave.h -- one wave computes the reverse-mode derivative of one
// lower Cholesky factorization.
//
// Not in the paper (which has no differentiation); the formula is the
// standard adjoint of A = L L^T (S. P. Smith 1995; I. Murray 2016):
//   P = Phi(L^T tril(Lbar))    (lower triangle, diagonal halved)
//   S = L^{-T} P L^{-1}
//   Abar = (S + S^T) / 2       (symmetric gradient)
// computed here with two right-side triangular solves in 16 x 16 FP64 MFMA
// tiles -- the right-variant solve the paper builds its trsm and Cholesky
// kernels on (Sec. 3.1.3): Z L = P gives Z = P L^{-1} (lower, since P and
// L^{-1} are), then W L = Z^T gives W = Z^T L^{-1} = S^T, and
// Abar = (W + W^T) / 2.  Each solve sweeps the block columns J from the
// right: tile(I,J) = (rhs(I,J) - sum_{K>J} X(I,K) L(K,J)) L_JJ^{-1}, with
// L_JJ^{-1} formed in registers (product of inverted column factors) and
// applied as an MFMA product.  Abar's storage is the workspace: P, then Z,
// then W overwrite it in an order that never reads a tile after it was
// replaced.
//
// Tiles are in accumulator order (lane (g, i), register r holds element
// (i, g + 4r) of the tile), as in potrf_wave.h; a transposed tile is loaded
// by swapping the element coordinates.
#pragma once

#include <utility>

#include "potrf_wave.h"

namespace mb {

struct AdjSmem {
    double t[16][17];  // tile transpose staging
};

// The 16 x 16 block M with M[i][c] = X(R0 + i, C0 + c), or X(C0 + c, R0 + i)
// when trans, in accumulator order.  Elements outside the n x n matrix read
// 0 (1 on the diagonal when ident); with lower, elements of X above its
// diagonal read 0.
__device__ __forceinline__ d4 adj_ld(const MB_GLOBAL double *X, size_t ld, int n, int R0, int C0,
                                     bool trans, bool lower, bool ident, int lr, int lg)
{
    d4 t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int c = lg + 4 * r;
        const int row = trans ? C0 + c : R0 + lr;
        const int col = trans ? R0 + lr : C0 + c;
        double v;
        if (row < n && col < n)
            v = (lower && row < col) ? 0.0 : X[(size_t)row + (size_t)col * ld];
        else
            v = (ident && row == col) ? 1.0 : 0.0;
        t[r] = v;
    }
    return t;
}

// Store M (accumulator order) to X(R0 + i, C0 + c), or X(C0 + c, R0 + i) when
// trans, inside the n x n matrix only.
__device__ __forceinline__ void adj_st(MB_GLOBAL double *X, size_t ld, int n, int R0, int C0,
                                       bool trans, const d4 &t, int lr, int lg)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int c = lg + 4 * r;
        const int row = trans ? C0 + c : R0 + lr;
        const int col = trans ? R0 + lr : C0 + c;
        if (row < n && col < n)
            X[(size_t)row + (size_t)col * ld] = t[r];
    }
}

// acc + sign * X Y^T for tiles in accumulator order.
__device__ __forceinline__ d4 adj_xyT(d4 acc, const d4 &x, const d4 &y, double sign)
{
#pragma unroll
    for (int s = 0; s < 4; ++s)
        acc = mfma16(sign * y[s], x[s], acc);
    return acc;
}

// Step C of the inverse of a lower-triangular tile t (accumulator order,
// nonzero diagonal): X <= C_C^{-1} X, where C_C is the identity with column C
// replaced by column C of t -- row C of X is divided by t_CC and the rows
// below lose t_iC / t_CC times it (rows above have t_iC = 0).  Both are one
// fma with row C of X, which sits in the same register of lane C of each
// group of 16 (a DPP broadcast); t_iC comes through the crossbar, t_CC from
// lane C; the reciprocal is the hardware estimate refined by Newton-Raphson.
template <int C>
__device__ __forceinline__ void inv_step(const d4 &t, d4 &x, int lane)
{
    constexpr int RC = C >> 2, GC = C & 3;
    // opaque lane index: the lane mask is formed here, not hoisted
    asm volatile("" : "+v"(lane));
    const int i = lane & 15;
    const double lic = lane_read(t[RC], 16 * GC + i);  // t[i][C]
    const double rinv = rcp_nr(row_bcast<C>(lic));    // 1 / t[C][C]
    const double ms = (i == C) ? 1.0 - rinv : lic * rinv;
    d4 xb;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        xb[r] = row_bcast<C>(x[r]);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        x[r] = fma(-ms, xb[r], x[r]);
}

template <int... C>
__device__ __forceinline__ void inv_steps(const d4 &t, d4 &x, int lane,
                                          std::integer_sequence<int, C...>)
{
    (inv_step<C>(t, x, lane), ...);
}

// Inverse of a lower-triangular tile t (accumulator order, nonzero
// diagonal): X = C_15^{-1} ... C_0^{-1} (inv_step), no LDS.
__device__ __forceinline__ d4 adj_inv_lower(const d4 &t, int lane)
{
    const int i = lane & 15, g = lane >> 4;
    d4 x;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        x[r] = (i == g + 4 * r) ? 1.0 : 0.0;
    inv_steps(t, x, lane, std::make_integer_sequence<int, 16>{});
    return x;
}

// Transpose of a tile in accumulator order, through LDS.
__device__ __forceinline__ d4 adj_transpose(const d4 &x, AdjSmem &S, int lane)
{
    const int i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        S.t[i][g + 4 * r] = x[r];
    wave_lds_sync();
    d4 y;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        y[r] = S.t[g + 4 * r][i];
    wave_lds_sync();
    return y;
}

// adj_ld with trans: the mirrored block loaded in its own order (consecutive
// lanes read consecutive rows of a column -- one cache line per 16 lanes)
// and transposed through LDS.  Reading the transposed elements directly puts
// 16 cache lines under every load instruction, which saturated the address
// units.
__device__ __forceinline__ d4 adj_ldt(const MB_GLOBAL double *X, size_t ld, int n, int R0, int C0,
                                      bool lower, bool ident, AdjSmem &S, int lane)
{
    return adj_transpose(adj_ld(X, ld, n, C0, R0, false, lower, ident, lane & 15, lane >> 4), S,
                         lane);
}

// Make this wave's global stores visible to its own later loads.
__device__ __forceinline__ void adj_fence() { wave_mem_sync(); }

// Abar <= adjoint of the Cholesky factorization at L for the cotangent Lbar
// (lower triangles of L and Lbar are read; the whole n x n Abar is written).
// NT = ceil(n / 16).
__device__ __forceinline__ void potrf_adj_wave(const double *Lp, size_t ldl, const double *Lbp,
                                               size_t ldlb, double *Ap, size_t lda, int n, int NT,
                                               AdjSmem &S, int lane)
{
    const MB_GLOBAL double *L = global_ptr(Lp);
    const MB_GLOBAL double *Lb = global_ptr(Lbp);
    MB_GLOBAL double *Ab = global_ptr(Ap);
    const int lr = lane & 15, lg = lane >> 4;
    const d4 zero = d4{0.0, 0.0, 0.0, 0.0};

    // P(I,J) = Phi( sum_{K>=I} L(K,I)^T Lbar(K,J) ), I >= J
    for (int J = 0; J < NT; ++J) {
        for (int I = J; I < NT; ++I) {
            d4 acc = zero;
            for (int K = I; K < NT; ++K) {
                const d4 lt = adj_ldt(L, ldl, n, 16 * I, 16 * K, K == I, false, S, lane);
                const d4 bt = adj_ldt(Lb, ldlb, n, 16 * J, 16 * K, K == J, false, S, lane);
                acc = adj_xyT(acc, lt, bt, 1.0);
            }
            if (I == J) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = lg + 4 * r;
                    acc[r] = c > lr ? 0.0 : (c == lr ? 0.5 * acc[r] : acc[r]);
                }
            }
            adj_st(Ab, lda, n, 16 * I, 16 * J, false, acc, lr, lg);
        }
    }
    adj_fence();

    // Z L = P, Z lower: Z(I,J) = (P(I,J) - sum_{J<K<=I} Z(I,K) L(K,J)) L_JJ^{-1}
    for (int J = NT - 1; J >= 0; --J) {
        const d4 ljj = adj_ld(L, ldl, n, 16 * J, 16 * J, false, true, true, lr, lg);
        const d4 winv_t = adj_transpose(adj_inv_lower(ljj, lane), S, lane);  // L_JJ^{-T}
        for (int I = J; I < NT; ++I) {
            d4 acc = adj_ld(Ab, lda, n, 16 * I, 16 * J, false, false, false, lr, lg);
            for (int K = J + 1; K <= I; ++K) {
                const d4 z = adj_ld(Ab, lda, n, 16 * I, 16 * K, false, false, false, lr, lg);
                const d4 lt = adj_ldt(L, ldl, n, 16 * J, 16 * K, false, false, S, lane);
                acc = adj_xyT(acc, z, lt, -1.0);  // - Z(I,K) L(K,J)
            }
            adj_st(Ab, lda, n, 16 * I, 16 * J, false, adj_xyT(zero, acc, winv_t, 1.0), lr, lg);
        }
        adj_fence();
    }

    // W L = Z^T: W(I,J) = (Z(J,I)^T - sum_{K>J} W(I,K) L(K,J)) L_JJ^{-1}
    for (int J = NT - 1; J >= 0; --J) {
        const d4 ljj = adj_ld(L, ldl, n, 16 * J, 16 * J, false, true, true, lr, lg);
        const d4 winv_t = adj_transpose(adj_inv_lower(ljj, lane), S, lane);
        for (int I = 0; I < NT; ++I) {
            d4 acc = I <= J ? adj_ldt(Ab, lda, n, 16 * I, 16 * J, I == J, false, S, lane) : zero;
            for (int K = J + 1; K < NT; ++K) {
                const d4 w = adj_ld(Ab, lda, n, 16 * I, 16 * K, false, false, false, lr, lg);
                const d4 lt = adj_ldt(L, ldl, n, 16 * J, 16 * K, false, false, S, lane);
                acc = adj_xyT(acc, w, lt, -1.0);
            }
            adj_st(Ab, lda, n, 16 * I, 16 * J, false, adj_xyT(zero, acc, winv_t, 1.0), lr, lg);
        }
        adj_fence();
    }

    // Abar = (W + W^T) / 2
    for (int J = 0; J < NT; ++J) {
        for (int I = J; I < NT; ++I) {
            const d4 a = adj_ld(Ab, lda, n, 16 * I, 16 * J, false, false, false, lr, lg);
            const d4 b = adj_ldt(Ab, lda, n, 16 * I, 16 * J, false, false, S, lane);
            d4 s;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                s[r] = 0.5 * (a[r] + b[r]);
            adj_st(Ab, lda, n, 16 * I, 16 * J, false, s, lr, lg);
            if (I != J)  // the mirrored block, stored in its own order
                adj_st(Ab, lda, n, 16 * J, 16 * I, false, adj_transpose(s, S, lane), lr, lg);
        }
    }
}

// The same adjoint for orders up to 16 NT (NT <= 4) with every tile in
// registers: L^T and Lbar^T are read once (coalesced, transposed through
// LDS), P and Z never leave the registers, the diagonal inverses are formed
// once for both solves, and Abar is written once -- no fences, no tile read
// back.  Tile indices are compile-time constants (NT is a template
// parameter), so the tile arrays are registers; tiles past the order are
// zero, the diagonal tiles of L padded with the identity.
template <int NT>
__device__ __forceinline__ void potrf_adj_regs(const double *Lp, size_t ldl, const double *Lbp,
                                               size_t ldlb, double *Ap, size_t lda, int n,
                                               AdjSmem &S, int lane)
{
    const MB_GLOBAL double *L = global_ptr(Lp);
    const MB_GLOBAL double *Lb = global_ptr(Lbp);
    MB_GLOBAL double *Ab = global_ptr(Ap);
    const int lr = lane & 15, lg = lane >> 4;
    const d4 zero = d4{0.0, 0.0, 0.0, 0.0};
    d4 LT[NT][NT];  // LT[K][I] = L(K,I)^T, K >= I
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int K = I; K < NT; ++K)
            LT[K][I] = adj_ldt(L, ldl, n, 16 * I, 16 * K, K == I, K == I, S, lane);

    // P(I,J) = Phi( sum_{K>=I} L(K,I)^T Lbar(K,J) ), I >= J, into Z
    d4 Z[NT][NT];
#pragma unroll
    for (int J = 0; J < NT; ++J) {
        d4 LbT[NT];
#pragma unroll
        for (int K = J; K < NT; ++K)
            LbT[K] = adj_ldt(Lb, ldlb, n, 16 * J, 16 * K, K == J, false, S, lane);
#pragma unroll
        for (int I = J; I < NT; ++I) {
            d4 acc = zero;
#pragma unroll
            for (int K = I; K < NT; ++K)
                acc = adj_xyT(acc, LT[K][I], LbT[K], 1.0);
            if (I == J) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = lg + 4 * r;
                    acc[r] = c > lr ? 0.0 : (c == lr ? 0.5 * acc[r] : acc[r]);
                }
            }
            Z[I][J] = acc;
        }
    }

    // L_JJ^{-T}, once for both solves
    d4 WT[NT];
#pragma unroll
    for (int J = 0; J < NT; ++J)
        WT[J] = adj_transpose(adj_inv_lower(adj_transpose(LT[J][J], S, lane), lane), S, lane);

    // Z L = P: Z(I,J) = (P(I,J) - sum_{J<K<=I} Z(I,K) L(K,J)) L_JJ^{-1}
#pragma unroll
    for (int J = NT - 1; J >= 0; --J) {
#pragma unroll
        for (int I = J; I < NT; ++I) {
            d4 acc = Z[I][J];
#pragma unroll
            for (int K = J + 1; K <= I; ++K)
                acc = adj_xyT(acc, Z[I][K], LT[K][J], -1.0);
            Z[I][J] = adj_xyT(zero, acc, WT[J], 1.0);
        }
    }

    // W L = Z^T: W(I,J) = (Z(J,I)^T - sum_{K>J} W(I,K) L(K,J)) L_JJ^{-1}
    d4 W[NT][NT];
#pragma unroll
    for (int J = NT - 1; J >= 0; --J) {
#pragma unroll
        for (int I = 0; I < NT; ++I) {
            d4 acc = I <= J ? adj_transpose(Z[J][I], S, lane) : zero;
#pragma unroll
            for (int K = J + 1; K < NT; ++K)
                acc = adj_xyT(acc, W[I][K], LT[K][J], -1.0);
            W[I][J] = adj_xyT(zero, acc, WT[J], 1.0);
        }
    }

    // Abar = (W + W^T) / 2, each block and its mirror stored in their own order
#pragma unroll
    for (int J = 0; J < NT; ++J) {
#pragma unroll
        for (int I = J; I < NT; ++I) {
            const d4 b = adj_transpose(W[J][I], S, lane);
            d4 s;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                s[r] = 0.5 * (W[I][J][r] + b[r]);
            adj_st(Ab, lda, n, 16 * I, 16 * J, false, s, lr, lg);
            if (I != J)
                adj_st(Ab, lda, n, 16 * J, 16 * I, false, adj_transpose(s, S, lane), lr, lg);
        }
    }
}

}  // namespace mb
