// gemm_regtile.h -- one wave computes one register tile of a dgemm straight
// from global memory (no LDS): the GPU form of the paper's no-pack variant
// 'D' (Sec. 2.2), extended by MFMA register blocking.  Used by the fused
// persistent kernel (fused.hip) and by the batched register-tile kernels
// (gemm_regtile.hip), which serve thin and flat shapes: a tile reads just the
// rows of op(A) and columns of op(B) it needs, so with TM = 1 (m <= 16) the
// large operand B is streamed exactly once, the GPU counterpart of the
// paper's observation that packing only the small operand (variants 'C' /
// 'Ct', Sec. 2.3.2) is best for rectangular results.
//
// Within one wave the operand fragments of a 16-deep k chunk partition the A
// and B panels exactly (lane (g, i) holds four k of row i, the four lane
// groups together all 16), so LDS would only add traffic.  As in the packed
// kernels the MFMA takes op(B) as its left operand and accumulates C^T, so a
// lane owns whole rows of C and the epilogue stores are coalesced along
// columns.
#pragma once

#include "mb_internal.h"

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

}  // namespace mb
