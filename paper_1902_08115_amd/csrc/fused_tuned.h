// fused_tuned.h -- cost model and tile rule of the fused uneven batch.
//
// Written by paper_1902_08115_amd/autotune.py (--fused) from measurements on
// MI355X: homogeneous batches of each task kind are timed through the fused
// kernel, and the wave time of one task (time x resident waves / tasks) is
// fitted as
//   dgemm tile   F + T * TM * TN + chunks * (M * TM * TN + L * (TM + TN))
//   dpotrf       P0 + P1 * nt + P2 * nt^2 + P3 * nt^3
//   adjoint      the same cubic with its own coefficients
// with chunks = ceil(k / 16) and nt = ceil(n / 16); a side of the register
// tile uses two 16-row MFMA blocks when that dimension exceeds kFusedTwoMin
// (chosen by timing the uneven batch).  Estimates order the work (longest
// first) and balance the per-XCD queues; they never change results.
#pragma once

namespace mb {

constexpr double kFusedGemmFixedNs = 3691.9;
constexpr double kFusedGemmTileNs = 676.5;
constexpr double kFusedGemmMfmaNs = 336.1;
constexpr double kFusedGemmLoadNs = 634.8;
constexpr double kFusedPotrfNs[4] = {4616.6, 11500.8, -1022.2, 247.7};
constexpr double kFusedAdjointNs[4] = {-19212.6, 56025.4, -13507.1, 3107.5};
constexpr double kFusedLasetNs = 2000.0;
constexpr int kFusedTwoMin = 16;
// waves of a 4-wave workgroup that start on the dpotrf class:
// round(4 * min(1, share * kFusedPotrfShareScale)), share = that class's
// estimated fraction of the work (measured best split on the uneven batch)
constexpr double kFusedPotrfShareScale = 1.802;

}  // namespace mb
