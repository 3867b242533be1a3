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
kernel menu of this library.  A class keeps the choice of the committed
gemm_tuned.h while that choice is within --keep-within (2%) of the fastest
candidate, so repeated runs do not reshuffle near-ties.  Needs a GPU:

  python -m paper_1902_08115_amd.autotune --out-dir out

With --fused it tunes the fused uneven batch instead and writes
fused_tuned.h: the wave time of every task kind is measured on homogeneous
plans (time x resident waves / tasks, i.e. under full load) and fitted to the
cost model the plan orders and balances work by, and the register-tile
threshold is chosen by timing the 100,000-problem uneven batch with each
candidate.
"""
from __future__ import annotations

import argparse
import gc
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


def header(table, skinny):
    def block(tab, indent):
        rows = []
        for t in TRANS:
            ent = ", ".join("{%d, %d}" % (v, c) for v, c in tab[t])
            rows.append(indent + "{" + ent + "},")
        return chr(10).join(rows)
    dims = ", ".join(str(x) if x < (1 << 30) else "1 << 30" for x in CLASS_MAX)
    sk = chr(10).join("    {" + chr(10) + block(skinny[c], "        ") + chr(10) + "    },"
                      for c in range(len(skinny)))
    return f"""// gemm_tuned.h -- size-class dispatch tables of the batched dgemm.
//
// Written by paper_1902_08115_amd/autotune.py from measurements on MI355X
// (square sweep and the thin / flat / small sweeps of every trans case); edit
// by re-running the tuner.
// Square table (m > 16 and n > 16): entry e for trans case (2*ta + tb)
// applies while max(m, n, k) <= kGemmTuneMaxDim[e].  Skinny tables
// kGemmSkinny[s]: s = 0 for m <= 16 and n <= 16 but not both <= 4 (class of
// k; the square sizes 8..16 and m = n = 16 with k above 16), s = 1 for
// m <= 16 < n (class of max(n, k)), s = 2 for n <= 16 < m (class of
// max(m, k)), s = 3 for m <= 4 and n <= 4 (class of k; m = n = 4).  A
// choice within 2% of the fastest candidate is kept from the previous
// table, so that run-to-run noise does not move it.  Variant 1 = direct kernel,
// 2 = packed kernel with the given configuration of the packed menu,
// 3 = register tiles (one 16-wide MFMA block per side of 16 or less, two
// otherwise).
#pragma once

namespace mb {{

constexpr int kGemmTuneEntries = {len(CLASS_MAX)};
constexpr int kGemmTuneMaxDim[kGemmTuneEntries] = {{{dims}}};
// {{variant, packed configuration}} per trans case and size class
constexpr int kGemmTune[4][kGemmTuneEntries][2] = {{
{block(table, "    ")}
}};

// {{variant, packed configuration}} per skinny class, trans case and size class
constexpr int kGemmSkinny[{len(skinny)}][4][kGemmTuneEntries][2] = {{
{sk}
}};

}}  // namespace mb
"""


def committed_tables(path):
    """The square and skinny tables of an existing gemm_tuned.h, as lists of
    {trans: [(variant, config) per class]} (None if it cannot be read)."""
    import re
    try:
        text = open(path).read()
    except OSError:
        return None, []
    def pairs(body):
        return [(int(a), int(b)) for a, b in re.findall(r"\{(-?\d+), (-?\d+)\}", body)]
    ne = len(CLASS_MAX)
    sq = re.search(r"kGemmTune\[4\]\[kGemmTuneEntries\]\[2\] = \{(.*?)\n\};", text, re.S)
    sk = re.search(r"kGemmSkinny\[(\d+)\]\[4\]\[kGemmTuneEntries\]\[2\] = \{(.*?)\n\};", text, re.S)
    if not sq or not sk or f"kGemmTuneEntries = {ne};" not in text:
        return None, []
    def split(p):
        return {t: p[i * ne:(i + 1) * ne] for i, t in enumerate(TRANS)}
    sqp, skp = pairs(sq.group(1)), pairs(sk.group(2))
    nsk = int(sk.group(1))
    if len(sqp) != 4 * ne or len(skp) != nsk * 4 * ne:
        return None, []
    return split(sqp), [split(skp[c * 4 * ne:(c + 1) * 4 * ne]) for c in range(nsk)]


def class_index(x):
    return next(i for i, cm in enumerate(CLASS_MAX) if x <= cm)


def fused_header(c):
    p = ", ".join("%.1f" % x for x in c["potrf"])
    a = ", ".join("%.1f" % x for x in c["adjoint"])
    return f"""// fused_tuned.h -- cost model and tile rule of the fused uneven batch.
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

namespace mb {{

constexpr double kFusedGemmFixedNs = {c["F"]:.1f};
constexpr double kFusedGemmTileNs = {c["T"]:.1f};
constexpr double kFusedGemmMfmaNs = {c["M"]:.1f};
constexpr double kFusedGemmLoadNs = {c["L"]:.1f};
constexpr double kFusedPotrfNs[4] = {{{p}}};
constexpr double kFusedAdjointNs[4] = {{{a}}};
constexpr double kFusedLasetNs = {c["laset"]:.1f};
constexpr int kFusedTwoMin = {c["two_min"]};
// waves of a 4-wave workgroup that start on the dpotrf class:
// round(4 * min(1, share * kFusedPotrfShareScale)), share = that class's
// estimated fraction of the work (measured best split on the uneven batch)
constexpr double kFusedPotrfShareScale = {c["share_scale"]:.3f};

}}  // namespace mb
"""


def fused_tune(args):
    import numpy as np
    import torch

    from paper_1902_08115_amd import _lib, blas, inputs
    waves = None
    rows = {"gemm": [], "potrf": [], "adjoint": [], "uneven": []}

    def run_plan(probs, restore=None, reps=args.reps, **opt):
        plan = blas.Plan(probs, **opt)
        st = plan.stats()
        best = 1e30
        for r in range(reps + 1):
            if restore is not None:
                restore()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.execute(blas.Plan.FUSED)
            e1.record()
            torch.cuda.synchronize()
            if r:
                best = min(best, e0.elapsed_time(e1))
        plan.close()
        return best, st

    # dgemm tiles: (TM, TN) from m, n around the threshold; k from 16 to 160
    for (m, n) in ((16, 16), (32, 32), (16, 32), (32, 16)):
        for k in (16, 32, 64, 128, 160):
            batch = min(60000, (1 << 30) // (8 * (m * k + k * n + m * n)))
            A = inputs.torch_colmajor(batch, m, k, seed=1)
            B = inputs.torch_colmajor(batch, k, n, seed=2)
            C = inputs.torch_colmajor(batch, m, n, seed=3)
            probs = [dict(op=0, transa="N", transb="N", m=m, n=n, k=k, lda=m, ldb=k, ldc=m,
                          alpha=1.0, beta=1.0, A=A.data_ptr() + 8 * m * k * b,
                          B=B.data_ptr() + 8 * k * n * b, C=C.data_ptr() + 8 * m * n * b)
                     for b in range(batch)]
            ms, st = run_plan(probs, tile_two_min=16)
            waves = st["workgroups"] * 4
            wt = ms * 1e6 * waves / st["units"]
            rows["gemm"].append((2 if m > 16 else 1, 2 if n > 16 else 1, (k + 15) // 16, wt))
            log(f"fused gemm {m}x{n}x{k}: {ms:.3f} ms, {wt:.0f} ns per tile")
            del A, B, C
    # dpotrf and adjoint
    for n in (16, 32, 48, 64, 96, 128, 160, 192, 256):
        batch = min(16384, (1 << 30) // (8 * n * n))
        M = inputs.torch_spd(batch, n, seed=5)
        X = M.clone()
        info = torch.zeros(batch, dtype=torch.int32, device="cuda")
        probs = [dict(op=1, uplo="L", n=n, ldc=n, C=X.data_ptr() + 8 * n * n * b,
                      info=info.data_ptr() + 4 * b) for b in range(batch)]
        ms, st = run_plan(probs, restore=lambda: X.copy_(M), potrf_waves=4)
        wt = ms * 1e6 * st["workgroups"] * 4 / st["units"]
        rows["potrf"].append(((n + 15) // 16, wt))
        log(f"fused potrf n={n}: {ms:.3f} ms, {wt:.0f} ns per task")
        Lb = inputs.torch_colmajor(batch, n, n, seed=6)
        Ab = torch.empty_like(Lb)
        probs = [dict(op=2, n=n, A=M.data_ptr() + 8 * n * n * b, lda=n,
                      B=Lb.data_ptr() + 8 * n * n * b, ldb=n, C=Ab.data_ptr() + 8 * n * n * b,
                      ldc=n) for b in range(batch)]
        # the adjoint of the factor of M: factor once, then time the adjoint
        X.copy_(M)
        assert _lib.dpotrf_strided_batched("L", n, X.data_ptr(), n, n * n, info.data_ptr(), batch,
                                           torch.cuda.current_stream().cuda_stream) == 0
        for p in probs:
            p["A"] = p["A"] - M.data_ptr() + X.data_ptr()
        ms, st = run_plan(probs, potrf_waves=4)
        wt = ms * 1e6 * st["workgroups"] * 4 / st["units"]
        rows["adjoint"].append(((n + 15) // 16, wt))
        log(f"fused adjoint n={n}: {ms:.3f} ms, {wt:.0f} ns per task")
        del M, X, Lb, Ab
    torch.cuda.empty_cache()

    # least squares on relative error (rows scaled by 1 / measured time), so
    # that short tasks are fitted as well as long ones
    g = np.array(rows["gemm"], dtype=float)
    tm, tn, ch, wt = g[:, 0], g[:, 1], g[:, 2], g[:, 3]
    X = np.stack([np.ones_like(tm), tm * tn, ch * tm * tn, ch * (tm + tn)], 1)
    F, T, Mc, Lc = np.linalg.lstsq(X / wt[:, None], np.ones_like(wt), rcond=None)[0]
    coef = {"F": F, "T": T, "M": Mc, "L": Lc}
    for kind in ("potrf", "adjoint"):
        q = np.array(rows[kind], dtype=float)
        V = np.stack([np.ones(len(q)), q[:, 0], q[:, 0] ** 2, q[:, 0] ** 3], 1)
        coef[kind] = list(np.linalg.lstsq(V / q[:, 1:2], np.ones(len(q)), rcond=None)[0])
    coef["laset"] = 2000.0

    # the tile threshold, timed on the uneven batch
    spec = inputs.uneven_spec(inputs.UNEVEN_COUNT, inputs.seed_for(3, 0))
    X0 = inputs.uneven_device(spec, inputs.seed_for(3, 200))
    Xw = X0.clone()
    info = torch.zeros(spec["count"], dtype=torch.int32, device="cuda")
    base = Xw.data_ptr()
    probs = []
    for i in range(spec["count"]):
        if spec["op"][i] == 0:
            probs.append(dict(op=0, transa="NT"[spec["ta"][i]], transb="NT"[spec["tb"][i]],
                              m=spec["m"][i], n=spec["n"][i], k=spec["k"][i], lda=spec["lda"][i],
                              ldb=spec["ldb"][i], ldc=spec["ldc"][i], alpha=1.0, beta=1.0,
                              A=base + 8 * int(spec["off_a"][i]), B=base + 8 * int(spec["off_b"][i]),
                              C=base + 8 * int(spec["off_c"][i])))
        else:
            probs.append(dict(op=1, uplo="L", n=spec["n"][i], ldc=spec["ldc"][i],
                              C=base + 8 * int(spec["off_c"][i]), info=info.data_ptr() + 4 * i))
    arr = _lib.problems_array(probs)
    best_t, best_ms = None, 1e30
    for t in (8, 16, 24, 32, 48):
        ms, _ = run_plan(arr, restore=lambda: Xw.copy_(X0), tile_two_min=t)
        rows["uneven"].append((t, ms))
        log(f"uneven batch, tile threshold {t}: {ms:.3f} ms")
        if ms < best_ms:
            best_t, best_ms = t, ms
    coef["two_min"] = best_t
    # the dpotrf class's share of the waves: the model's share of the work
    # scaled so that the plan's rule reproduces the best measured split
    tmv = np.where(spec["m"] > best_t, 2, 1)
    tnv = np.where(spec["n"] > best_t, 2, 1)
    gm = spec["op"] == 0
    tiles = np.ceil(spec["m"] / (16 * tmv)) * np.ceil(spec["n"] / (16 * tnv))
    chv = np.ceil(spec["k"] / 16)
    gem = float((tiles * (F + T * tmv * tnv + chv * (Mc * tmv * tnv + Lc * (tmv + tnv))))[gm].sum())
    ntv = np.ceil(spec["n"][~gm] / 16)
    pc = coef["potrf"]
    pot = float((pc[0] + pc[1] * ntv + pc[2] * ntv ** 2 + pc[3] * ntv ** 3).sum())
    share = pot / (pot + gem)
    best_w, best_ms = None, 1e30
    for w in (1, 2, 3):
        ms, _ = run_plan(arr, restore=lambda: Xw.copy_(X0), tile_two_min=best_t, potrf_waves=w)
        rows["uneven"].append(("potrf_waves", w, ms))
        log(f"uneven batch, dpotrf-class waves {w}: {ms:.3f} ms")
        if ms < best_ms:
            best_w, best_ms = w, ms
    coef["share_scale"] = best_w / (4.0 * share)
    log(f"model dpotrf share {share:.3f}; best waves {best_w}; scale {coef['share_scale']:.3f}")
    os.makedirs(args.out_dir, exist_ok=True)
    with open(os.path.join(args.out_dir, "fused_tuned.h"), "w") as f:
        f.write(fused_header(coef))
    with open(os.path.join(args.out_dir, "autotune_fused.json"), "w") as f:
        json.dump({"rows": rows, "coef": {k: (list(map(float, v)) if isinstance(v, list) else
                                              float(v)) for k, v in coef.items()},
                   "time": time.strftime("%Y-%m-%d %H:%M:%S")}, f, indent=1)
    log("wrote fused_tuned.h and autotune_fused.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out-dir", default=".")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--sizes", default=None)
    ap.add_argument("--fused", action="store_true", help="tune the fused uneven batch")
    ap.add_argument("--square-only", action="store_true", help="skip the thin / flat sweeps")
    ap.add_argument("--keep-within", type=float, default=0.02,
                    help="keep the committed choice when it is this close to the fastest")
    args = ap.parse_args()
    # no garbage collection inside the timed calls (a full collection stalls
    # the launching thread and would lengthen one candidate's time)
    gc.collect()
    gc.disable()
    if args.fused:
        fused_tune(args)
        return
    sizes = [int(x) for x in args.sizes.split(",")] if args.sizes else list(SIZES)

    import torch

    from paper_1902_08115_amd import _lib, inputs
    sh = torch.cuda.current_stream().cuda_stream
    ncfg = _lib.dgemm_config_count()
    names = [_lib.dgemm_config_name(c) for c in range(ncfg)]
    limit = [_lib.dgemm_config_max_mn(c) for c in range(ncfg)]
    results = []
    old_sq, old_sk = committed_tables(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                   "csrc", "gemm_tuned.h"))

    def incumbent(table, t, x):
        """The committed choice of class x in table (None: no such table)."""
        if table is None:
            return None
        v, c = table[t][class_index(x)]
        if v == 1:
            return "direct"
        if v == 3:
            return "regtile"
        return names[c] if 0 <= c < ncfg else None

    def measure(m, n, k, t, label, inc=None):
        """Time every applicable candidate on a ~1 GiB batch of (m, n, k); the
        committed choice inc is kept when it is within --keep-within of the
        fastest."""
        ar, ac = (m, k) if t[0] == "N" else (k, m)
        br, bc = (k, n) if t[1] == "N" else (n, k)
        batch = min(1 << 22, (1 << 30) // (8 * (m * k + k * n + m * n)))
        A = inputs.torch_colmajor(batch, ar, ac, seed=11)
        B = inputs.torch_colmajor(batch, br, bc, seed=12)
        C = inputs.torch_colmajor(batch, m, n, seed=13)
        pa, pb, pc = A.data_ptr(), B.data_ptr(), C.data_ptr()
        sA, sB, sC = ar * ac, br * bc, m * n
        cands = [("direct", 1, -1), ("regtile", 3, -1)] + [
            (names[c], 2, c) for c in range(ncfg) if limit[c] >= max(m, n)]
        timings = {}
        for name, var, cfg in cands:
            if cfg < 0:
                def fn(var=var):
                    st = _lib.dgemm_strided_batched(t[0], t[1], m, n, k, 1.0, pa, ar, sA, pb, br,
                                                    sB, 1.0, pc, m, sC, batch, sh, var)
                    assert st == 0, st
            else:
                def fn(cfg=cfg):
                    st = _lib.dgemm_strided_batched_config(t[0], t[1], m, n, k, 1.0, pa, ar, sA,
                                                           pb, br, sB, 1.0, pc, m, sC, batch,
                                                           cfg, sh)
                    assert st == 0, st
            timings[name] = time_call(torch, fn, args.reps)
        fastest = min(timings, key=timings.get)
        win = fastest
        if inc in timings and timings[inc] <= (1.0 + args.keep_within) * timings[fastest]:
            win = inc
        flops = 2.0 * m * n * k * batch
        results.append({"sweep": label, "m": m, "n": n, "k": k, "trans": t, "batch": batch,
                        "ms": timings, "best": win, "fastest": fastest, "incumbent": inc,
                        "best_gflops": flops / timings[win] / 1e6})
        log(f"{label} {m}x{n}x{k} {t}: best {win} {flops / timings[win] / 1e6:.0f} GF/s " + " ".join(
            f"{kk.replace('gemm_packed_', '')}={v:.3f}" for kk, v in timings.items()))
        del A, B, C
        torch.cuda.empty_cache()
        if win == "direct":
            return (1, -1)
        if win == "regtile":
            return (3, -1)
        return (2, names.index(win))

    def to_table(best):
        table = {}
        for t in TRANS:
            row = []
            for cm in CLASS_MAX:
                # a class is represented by the largest measured size inside it
                inside = [n for n in best[t] if n <= cm]
                n = max(inside) if inside else min(best[t])
                v, c = best[t][n]
                if cm > 320 and v == 2 and limit[c] < (1 << 30):
                    c = names.index("gemm_packed_tile64_k16")
                row.append((v, c))
            table[t] = row
        return table

    # the committed skinny tables: 4 classes, or the earlier 3 (no tiny class;
    # class 0 then held m = n = 4 for k above 16 and the square sizes below)
    old4 = len(old_sk) == 4
    inc_tiny = old_sk[3] if old4 else None
    square = {t: {} for t in TRANS}
    skinny = [{t: {} for t in TRANS} for _ in range(4)]
    for n in sizes:
        for t in TRANS:
            if n > 16:
                square[t][n] = measure(n, n, n, t, "square", incumbent(old_sq, t, n))
            elif n <= 4:   # m, n <= 4: the tiny table
                inc = incumbent(inc_tiny if old4 else (old_sk[0] if old_sk else None), t, n)
                skinny[3][t][n] = measure(n, n, n, t, "square", inc)
            else:          # m, n <= 16: the small table
                inc = incumbent(old_sk[0] if old_sk else None, t, n)
                skinny[0][t][n] = measure(n, n, n, t, "square", inc)
    if not args.square_only:
        for s in [x for x in sizes if x > 4]:
            for t in TRANS:
                if s <= 16:  # m = n = 4 with short k (square sizes above 4 are 8..16)
                    skinny[3][t][s] = measure(4, 4, s, t, "m=n=4", incumbent(inc_tiny, t, s))
                    continue
                inc = incumbent(inc_tiny if old4 else (old_sk[0] if old_sk else None), t, s)
                skinny[3][t][s] = measure(4, 4, s, t, "m=n=4", inc)
                skinny[0][t][s] = measure(16, 16, s, t, "m=n=16",
                                          incumbent(old_sk[0] if old4 else None, t, s))
                skinny[1][t][s] = measure(4, s, s, t, "m=4",
                                          incumbent(old_sk[1] if old_sk else None, t, s))
                skinny[2][t][s] = measure(s, 4, s, t, "n=4",
                                          incumbent(old_sk[2] if old_sk else None, t, s))
    for t in TRANS:  # classes below every measured size take the smallest measured one
        for d in [square] + skinny:
            if not d[t]:
                d[t] = {16: (3, -1)}
    table = to_table(square)
    sk = [to_table(skinny[c]) for c in range(4)]
    os.makedirs(args.out_dir, exist_ok=True)
    with open(os.path.join(args.out_dir, "gemm_tuned.h"), "w") as f:
        f.write(header(table, sk))
    with open(os.path.join(args.out_dir, "autotune.json"), "w") as f:
        json.dump({"configs": names, "results": results,
                   "time": time.strftime("%Y-%m-%d %H:%M:%S")}, f, indent=1)
    log("wrote gemm_tuned.h and autotune.json")


if __name__ == "__main__":
    main()
