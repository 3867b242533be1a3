"""Autotuner for the batched dgemm size switch and packed tile configurations.

For every trans case and every size class of the square benchmark sweep it
times the direct kernel and each packed configuration that can hold the
problem, on the benchmark's own batch sizes (about 1 GiB of A + B + C, inputs
resident in device memory), and writes

  * gemm_tuned.h   -- the dispatch table compiled into the library
                      (which family, which packed configuration, per class);
  * autotune.json  -- every measurement.

This is the paper's variant switching (Sec. 2.4: the switching point is found
by measurement and differs per routine and architecture) applied to the
kernel menu of this library.  Needs a GPU:

  python -m paper_1902_08115_amd.autotune --out-dir gpurun_out
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

SIZES = (4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 300)
CLASS_MAX = (4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 320, 1 << 30)
TRANS = ("NN", "NT", "TN", "TT")


def log(msg):
    print(f"[autotune] {msg}", file=sys.stderr, flush=True)


def time_call(torch, fn, reps):
    for _ in range(2):
        fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def header(table):
    rows = []
    for t in TRANS:
        ent = ", ".join("{%d, %d}" % (v, c) for v, c in table[t])
        rows.append("    {" + ent + "},")
    dims = ", ".join(str(x) if x < (1 << 30) else "1 << 30" for x in CLASS_MAX)
    return f"""// gemm_tuned.h -- size-class dispatch table of the batched dgemm.
//
// Written by paper_1902_08115_amd/autotune.py from measurements on MI355X
// (square batched sweep, every trans case); edit by re-running the tuner.
// Entry e of the table for trans case (2*ta + tb) applies while
// max(m, n, k) <= kGemmTuneMaxDim[e]; variant 1 = direct kernel, 2 = packed
// kernel with the given configuration of the packed menu.
#pragma once

namespace mb {{

constexpr int kGemmTuneEntries = {len(CLASS_MAX)};
constexpr int kGemmTuneMaxDim[kGemmTuneEntries] = {{{dims}}};
// {{variant, packed configuration}} per trans case and size class
constexpr int kGemmTune[4][kGemmTuneEntries][2] = {{
{chr(10).join(rows)}
}};

}}  // namespace mb
"""


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out-dir", default=".")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--sizes", default=None)
    args = ap.parse_args()
    sizes = [int(x) for x in args.sizes.split(",")] if args.sizes else list(SIZES)

    import torch

    from paper_1902_08115_amd import _lib, inputs
    sh = torch.cuda.current_stream().cuda_stream
    ncfg = _lib.dgemm_config_count()
    names = [_lib.dgemm_config_name(c) for c in range(ncfg)]
    limit = [_lib.dgemm_config_max_mn(c) for c in range(ncfg)]
    results = []
    best = {t: {} for t in TRANS}
    for n in sizes:
        batch = inputs.gemm_sweep_batch(n)
        A = inputs.torch_colmajor(batch, n, n, seed=11)
        B = inputs.torch_colmajor(batch, n, n, seed=12)
        C = inputs.torch_colmajor(batch, n, n, seed=13)
        pa, pb, pc = A.data_ptr(), B.data_ptr(), C.data_ptr()
        for t in TRANS:
            cands = [("direct", None)] + [(names[c], c) for c in range(ncfg) if limit[c] >= n]
            timings = {}
            for name, cfg in cands:
                if cfg is None:
                    def fn():
                        st = _lib.dgemm_strided_batched(t[0], t[1], n, n, n, 1.0, pa, n, n * n,
                                                        pb, n, n * n, 1.0, pc, n, n * n, batch,
                                                        sh, _lib.VARIANT_DIRECT)
                        assert st == 0, st
                else:
                    def fn(cfg=cfg):
                        st = _lib.dgemm_strided_batched_config(t[0], t[1], n, n, n, 1.0, pa, n,
                                                               n * n, pb, n, n * n, 1.0, pc, n,
                                                               n * n, batch, cfg, sh)
                        assert st == 0, st
                timings[name] = time_call(torch, fn, args.reps)
            win = min(timings, key=timings.get)
            best[t][n] = (1, -1) if win == "direct" else (2, names.index(win))
            flops = 2.0 * n ** 3 * batch
            results.append({"n": n, "trans": t, "batch": batch, "ms": timings, "best": win,
                            "best_gflops": flops / timings[win] / 1e6})
            log(f"n={n} {t}: best {win} {flops / timings[win] / 1e6:.0f} GF/s "
                + " ".join(f"{k.replace('gemm_packed_', '')}={v:.3f}" for k, v in timings.items()))
        del A, B, C
        torch.cuda.empty_cache()

    table = {}
    for t in TRANS:
        row = []
        for cm in CLASS_MAX:
            # the class is represented by the largest measured size inside it
            inside = [n for n in best[t] if n <= cm]
            n = max(inside) if inside else min(best[t])
            v, c = best[t][n]
            if cm > 320 and v == 2 and limit[c] < (1 << 30):
                c = names.index("gemm_packed_tile64_k16")
            row.append((v, c))
        table[t] = row
    os.makedirs(args.out_dir, exist_ok=True)
    with open(os.path.join(args.out_dir, "gemm_tuned.h"), "w") as f:
        f.write(header(table))
    with open(os.path.join(args.out_dir, "autotune.json"), "w") as f:
        json.dump({"configs": names, "results": results,
                   "time": time.strftime("%Y-%m-%d %H:%M:%S")}, f, indent=1)
    log("wrote gemm_tuned.h and autotune.json")


if __name__ == "__main__":
    main()
