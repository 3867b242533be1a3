// gemm_tuned.h -- size-class dispatch table of the batched dgemm.
//
// Written by paper_1902_08115_amd/autotune.py from measurements on MI355X
// (square batched sweep, every trans case); edit by re-running the tuner.
// Entry e of the table for trans case (2*ta + tb) applies while
// max(m, n, k) <= kGemmTuneMaxDim[e]; variant 1 = direct kernel, 2 = packed
// kernel with the given configuration of the packed menu.
#pragma once

namespace mb {

constexpr int kGemmTuneEntries = 14;
constexpr int kGemmTuneMaxDim[kGemmTuneEntries] = {4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 320, 1 << 30};
// {variant, packed configuration} per trans case and size class
constexpr int kGemmTune[4][kGemmTuneEntries][2] = {
    {{1, -1}, {1, -1}, {2, 0}, {2, 0}, {2, 1}, {2, 1}, {2, 2}, {2, 4}, {2, 6}, {2, 3}, {2, 3}, {2, 3}, {2, 5}, {2, 5}},
    {{1, -1}, {1, -1}, {2, 0}, {2, 0}, {2, 1}, {2, 1}, {2, 2}, {2, 3}, {2, 6}, {2, 3}, {2, 3}, {2, 5}, {2, 5}, {2, 5}},
    {{1, -1}, {2, 0}, {2, 0}, {2, 0}, {2, 1}, {2, 1}, {2, 2}, {2, 3}, {2, 6}, {2, 3}, {2, 3}, {2, 10}, {2, 5}, {2, 5}},
    {{1, -1}, {2, 0}, {2, 0}, {2, 0}, {2, 1}, {2, 1}, {2, 2}, {2, 3}, {2, 6}, {2, 3}, {2, 3}, {2, 5}, {2, 5}, {2, 5}},
};

}  // namespace mb
