// fused_tuned.h -- cost model and tile rule of the fused uneven batch.
//
// Written by paper_1902_08115_amd/autotune.py (--fused) from measurements on
// MI355X: homogeneous batches of each unit type are timed through the fused
// kernel, and the wave time of one unit is fitted as
//   dgemm tile   F + T * TM * TN + chunks * (M * TM * TN + L * (TM + TN))
//   dpotrf       P0 + P1 * nt + P2 * nt^2 + P3 * nt^3
// with chunks = ceil(k / 16) and nt = ceil(n / 16); a side of the register
// tile uses two 16-row MFMA blocks when that dimension exceeds kFusedTwoMin.
// Estimates order the work (longest first) and balance the per-XCD queues;
// they never change results.
#pragma once

namespace mb {

constexpr double kFusedGemmFixedNs = 1600.0;
constexpr double kFusedGemmTileNs = 1800.0;
constexpr double kFusedGemmMfmaNs = 80.0;
constexpr double kFusedGemmLoadNs = 50.0;
constexpr double kFusedPotrfNs[4] = {525.0, 13500.0, -607.0, 144.0};
constexpr double kFusedAdjointNs[4] = {1500.0, 40000.0, 0.0, 450.0};
constexpr double kFusedLasetNs = 2000.0;
constexpr int kFusedTwoMin = 16;

}  // namespace mb
