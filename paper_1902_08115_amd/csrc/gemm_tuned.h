// gemm_tuned.h -- size-class dispatch tables of the batched dgemm.
//
// Written by paper_1902_08115_amd/autotune.py from measurements on MI355X
// (square sweep and the thin / flat / small sweeps of every trans case); edit
// by re-running the tuner.
// Square table (m > 16 and n > 16): entry e for trans case (2*ta + tb)
// applies while max(m, n, k) <= kGemmTuneMaxDim[e].  Skinny tables
// kGemmSkinny[s]: s = 0 for m <= 16 and n <= 16 (class of k; the square
// sizes up to 16 fall here), s = 1 for m <= 16 < n (class of max(n, k)),
// s = 2 for n <= 16 < m (class of max(m, k)).  Variant 1 = direct kernel,
// 2 = packed kernel with the given configuration of the packed menu,
// 3 = register tiles (one 16-wide MFMA block per side of 16 or less, two
// otherwise).
#pragma once

namespace mb {

constexpr int kGemmTuneEntries = 14;
constexpr int kGemmTuneMaxDim[kGemmTuneEntries] = {4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 320, 1 << 30};
// {variant, packed configuration} per trans case and size class
constexpr int kGemmTune[4][kGemmTuneEntries][2] = {
    {{3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {2, 3}, {3, -1}, {2, 11}, {2, 13}, {2, 5}, {2, 15}, {2, 5}, {2, 5}},
    {{3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {2, 1}, {2, 3}, {3, -1}, {2, 6}, {2, 15}, {2, 5}, {2, 15}, {2, 5}, {2, 5}},
    {{2, 1}, {2, 1}, {2, 1}, {2, 1}, {2, 1}, {2, 2}, {2, 3}, {2, 5}, {2, 11}, {2, 3}, {2, 3}, {2, 15}, {2, 5}, {2, 5}},
    {{2, 1}, {2, 1}, {2, 1}, {2, 1}, {2, 1}, {2, 1}, {2, 3}, {2, 4}, {2, 6}, {2, 15}, {2, 5}, {2, 15}, {2, 5}, {2, 5}},
};

// {variant, packed configuration} per skinny class, trans case and size class
constexpr int kGemmSkinny[3][4][kGemmTuneEntries][2] = {
    {
        {{1, -1}, {2, 0}, {2, 0}, {2, 0}, {3, -1}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {3, -1}, {3, -1}},
        {{1, -1}, {1, -1}, {2, 0}, {2, 0}, {1, -1}, {1, -1}, {1, -1}, {1, -1}, {1, -1}, {1, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}},
        {{1, -1}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {3, -1}, {3, -1}},
        {{1, -1}, {2, 0}, {2, 0}, {2, 0}, {3, -1}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {2, 0}, {3, -1}, {3, -1}},
    },
    {
        {{3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}},
        {{3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}},
        {{3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {2, 1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}},
        {{3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}},
    },
    {
        {{3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}},
        {{3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}},
        {{3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}},
        {{3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}, {3, -1}},
    },
};

}  // namespace mb
