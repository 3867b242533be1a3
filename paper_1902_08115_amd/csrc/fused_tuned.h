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

constexpr double kFusedGemmFixedNs = 3582.3;
constexpr double kFusedGemmTileNs = 759.8;
constexpr double kFusedGemmMfmaNs = 320.2;
constexpr double kFusedGemmLoadNs = 649.3;
constexpr double kFusedPotrfNs[4] = {2874.5, 13981.2, -1322.2, 273.4};
constexpr double kFusedAdjointNs[4] = {-2548.8, 68865.4, -17597.5, 3372.1};
constexpr double kFusedLasetNs = 2000.0;
constexpr int kFusedTwoMin = 16;
// waves of a 4-wave workgroup that start on the dpotrf class:
// round(4 * min(1, share * kFusedPotrfShareScale)), share = that class's
// estimated fraction of the work (measured best split on the uneven batch)
constexpr double kFusedPotrfShareScale = 1.721;

}  // namespace mb
