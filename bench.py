#!/usr/bin/env python3
"""Batched FP64 dgemm / dpotrf('L') throughput on one MI355X.

One step is one pass of the whole hot path over resident synthetic inputs:
  * the square dgemm sweep, m = n = k in {4, 8, 12, 16, 24, 32, 48, 64, 96,
    128, 192, 256, 300}, all four trans cases, alpha = beta = 1, lda = m,
    batch per size such that A + B + C hold about 1 GiB, strided contiguous;
  * the dpotrf 'L' sweep, n in {8, 16, 32, 64, 128, 192, 256}, batch 4096,
    A = M M^T + n I with one non-SPD instance (a_jj = -1) per size.
Every call goes through the C ABI of libmi355blas.so on torch's current
stream; per-launch durations come from events recorded on that stream.

Prints ONE compact JSON line on stdout (the headline, the dominant kernel's
roofline, the CPU baseline, GFLOP/s against n); progress goes to stderr, and
so does the full record (per size, per kernel class, the uneven-batch,
differentiation and Riccati workloads) as one `[bench] details {...}` line,
also written to --details-out when given.

  python bench.py [--gpus 1] [--steps K] [--warmup W]
  python bench.py --crossover     # direct vs packed dgemm at every sweep size
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "batched FP64 GFLOP/s vs n (dgemm, dpotrf) & % FP64 peak; fused vs plain"
PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (vector and matrix)
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E
RIDGE = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gemm_work(n, batch):
    """(flops, algorithmic bytes) of one square call with beta != 0."""
    return 2.0 * n ** 3 * batch, 8.0 * 4 * n * n * batch


def potrf_work(n, batch):
    """(flops n^3/3, bytes: lower triangle read + written, plus info)."""
    return n ** 3 / 3.0 * batch, 8.0 * n * (n + 1) * batch + 4.0 * batch


class Timer:
    """Per-launch event pairs on the launch stream."""

    def __init__(self, torch):
        self.torch = torch
        self.rec = []

    def around(self, key, fn):
        t = self.torch
        e0 = t.cuda.Event(enable_timing=True)
        e1 = t.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        self.rec.append((key, e0, e1))

    def collect(self):
        out = {}
        for key, e0, e1 in self.rec:
            out.setdefault(key, []).append(e0.elapsed_time(e1))
        self.rec = []
        return out


def source_digest(paths):
    h = hashlib.sha256()
    for p in sorted(paths):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def riccati_kernel_label(nx, nu):
    """The kernel the library runs for a Riccati shape (csrc/riccati.hip)."""
    m = nx + nu
    if m <= 16:
        return "riccati_small_kernel"
    if m <= 96 and 1 <= nx <= 64:
        return f"riccati_regs_kernel<{(m + 15) // 16},{(nx + 15) // 16}>"
    if ((m + 15) // 16) * ((nx + 15) // 16) <= 6:
        return "riccati_kernel<6> (C in LDS)"
    return "riccati_kernel<0> (C in the workspace)"


def traffic_for(kernel, per_launch_bytes):
    """HBM traffic measured with rocprofv3 counters for this kernel, if the
    committed measurement was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except Exception:
        return None
    ent = data.get(kernel)
    if not ent:
        return None
    csrc = os.path.join(ROOT, "paper_1902_08115_amd", "csrc")
    names = ent.get("sources") or [f for f in os.listdir(csrc) if f.endswith((".hip", ".h"))]
    srcs = [os.path.join(csrc, f) for f in names]
    if not all(os.path.exists(p) for p in srcs) or ent.get("source_digest") != source_digest(srcs):
        return None
    return ent.get("bytes_per_launch")


def build_inputs(torch, inputs, args):
    gemm = []
    for si, n in enumerate(args.gemm_sizes):
        batch = inputs.gemm_sweep_batch(n)
        s = inputs.seed_for(1, inputs.GEMM_SWEEP_SIZES.index(n))
        A = inputs.torch_colmajor(batch, n, n, seed=s)
        B = inputs.torch_colmajor(batch, n, n, seed=s + 1)
        C = inputs.torch_colmajor(batch, n, n, seed=s + 2)
        gemm.append((n, batch, A, B, C))
    potrf = []
    for n in args.potrf_sizes:
        si = inputs.POTRF_SWEEP_SIZES.index(n)
        batch = args.potrf_batch
        master = inputs.torch_spd(batch, n, seed=inputs.seed_for(2, si))
        rs = np.random.Generator(np.random.PCG64(inputs.seed_for(2, si)))
        bad_b, bad_j = int(rs.integers(0, batch)), int(rs.integers(0, n))
        master[bad_b, bad_j, bad_j] = -1.0
        copies = [master.clone() for _ in range(args.copies)]
        info = torch.empty(batch, dtype=torch.int32, device="cuda")
        potrf.append((n, batch, master, copies, info, (bad_b, bad_j)))
    torch.cuda.synchronize()
    return gemm, potrf


def run_step(step, gemm, potrf, _lib, stream, timer, restore_counter):
    sh = stream.cuda_stream
    for (n, batch, A, B, C) in gemm:
        for trans in ("NN", "NT", "TN", "TT"):
            ta, tb = trans

            def call(ta=ta, tb=tb, n=n, batch=batch, A=A, B=B, C=C):
                st = _lib.dgemm_strided_batched(ta, tb, n, n, n, 1.0, A.data_ptr(), n, n * n,
                                                B.data_ptr(), n, n * n, 1.0, C.data_ptr(), n,
                                                n * n, batch, sh)
                if st != 0:
                    raise RuntimeError(f"mb_dgemm_strided_batched {trans} n={n}: status {st}")
            if timer is None:
                call()
            else:
                timer.around(("dgemm", trans, n), call)
    for (n, batch, master, copies, info, _) in potrf:
        c = step % len(copies)
        if step >= len(copies):  # this copy was factored before: restore it (inside the step)
            copies[c].copy_(master)
            restore_counter[0] += 2 * master.numel() * 8

        def callp(n=n, batch=batch, X=copies[c], info=info):
            st = _lib.dpotrf_strided_batched("L", n, X.data_ptr(), n, n * n, info.data_ptr(),
                                             batch, sh)
            if st != 0:
                raise RuntimeError(f"mb_dpotrf_strided_batched n={n}: status {st}")
        if timer is None:
            callp()
        else:
            timer.around(("dpotrf", "L", n), callp)


def ceilings(torch, _lib, stream):
    """Measured ceilings next to the published ones: FP64 matrix-core and
    vector-FMA loops (mb_ceiling_fp64, 4 waves per SIMD) and a 1 GiB
    device-to-device copy (read + write bytes), best of 3 event-timed runs."""
    sh = stream.cuda_stream
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = cus * 4
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    res = {"compute_units": cus}
    for key, kind, iters in (("fp64_mfma_tflops", 0, 20000), ("fp64_fma_tflops", 1, 100000)):
        best = None
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            st, fl = _lib.ceiling_fp64(kind, blocks, iters, out.data_ptr(), sh)
            e1.record()
            if st != 0:
                raise RuntimeError(f"mb_ceiling_fp64 kind {kind}: status {st}")
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        res[key] = round(fl / best / 1e9, 2)
    # HBM: the library's streaming probes (16-byte non-temporal accesses, four
    # loads in flight per thread) over 1 GiB per stream -- far beyond the
    # 256 MiB last-level cache -- at two grid sizes, best of 3 each; and
    # torch's device-to-device copy beside them
    n = 1 << 27
    src = torch.ones(3 * n, dtype=torch.float64, device="cuda")
    dst = torch.empty(n, dtype=torch.float64, device="cuda")
    part = torch.empty(cus * 32 * 256, dtype=torch.float64, device="cuda")
    for key, kind in (("hbm_read_gbps", 0), ("hbm_copy_gbps", 1), ("hbm_3r1w_gbps", 2)):
        best = None
        for blocks in (cus * 8, cus * 32):
            for _ in range(3):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                st, by = _lib.ceiling_hbm(kind, src.data_ptr(), dst.data_ptr(), n, blocks,
                                          part.data_ptr(), sh)
                e1.record()
                if st != 0:
                    raise RuntimeError(f"mb_ceiling_hbm kind {kind}: status {st}")
                torch.cuda.synchronize()
                rate = by / e0.elapsed_time(e1) / 1e6
                best = rate if best is None else max(best, rate)
        res[key] = round(best, 1)
    best = None
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src[:n])
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    res["torch_copy_gbps"] = round(2 * n * 8 / best / 1e6, 1)
    res["spec"] = {"fp64_tflops": PEAK_FP64_TFLOPS, "hbm_gbps": PEAK_HBM_GBS}
    del src, dst, out, part
    torch.cuda.empty_cache()
    return res


def potrf_hot(torch, _lib, potrf, stream, reps=7):
    """dpotrf with a hot input (the paper's protocol): one copy is restored
    from the pristine matrix right before each event-timed factorization (the
    restore is outside the events), so up to the cache sizes the input is
    resident when the factorization starts.  The sweep's own figure is the cold
    one: every step factors a copy that was last touched steps earlier."""
    sh = stream.cuda_stream
    out = {}
    for (n, batch, master, copies, info, _) in potrf:
        X = copies[0]
        ts = []
        for _ in range(reps):
            X.copy_(master)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            st = _lib.dpotrf_strided_batched("L", n, X.data_ptr(), n, n * n, info.data_ptr(),
                                             batch, sh)
            e1.record()
            if st != 0:
                raise RuntimeError(f"mb_dpotrf_strided_batched n={n}: status {st}")
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        fl, _ = potrf_work(n, batch)
        med = float(np.median(ts))
        out[n] = {"ms_median": round(med, 4), "ms_min": round(min(ts), 4),
                  "gflops": round(fl / med / 1e6, 1), "reps": reps}
    return out


def cpu_baseline(torch, oracle, gemm, potrf, flops_per_case):
    """The oracle on the host cores, on a bounded prefix of each case."""
    total_flops = 0.0
    total_time = 0.0
    parts = []
    for (n, batch, A, B, C) in gemm:
        cnt = int(max(1, min(batch, flops_per_case // (2 * n ** 3))))
        a = A[:cnt].transpose(1, 2).contiguous().cpu().numpy().ravel()
        b = B[:cnt].transpose(1, 2).contiguous().cpu().numpy().ravel()
        c0 = C[:cnt].transpose(1, 2).contiguous().cpu().numpy().ravel()
        for trans in ("NN", "NT", "TN", "TT"):
            c = c0.copy()
            t0 = time.perf_counter()
            oracle.dgemm_strided_batched(trans[0], trans[1], n, n, n, 1.0, a, n, n * n, b, n,
                                         n * n, 1.0, c, n, n * n, cnt)
            total_time += time.perf_counter() - t0
            total_flops += 2.0 * n ** 3 * cnt
        parts.append(f"dgemm n={n}: {cnt} instances x 4 trans")
    for (n, batch, master, copies, info, _) in potrf:
        cnt = int(max(1, min(batch, flops_per_case // max(1, n ** 3 // 3))))
        x = master[:cnt].transpose(1, 2).contiguous().cpu().numpy().ravel()
        t0 = time.perf_counter()
        oracle.dpotrf_l_strided_batched(n, x, n, n * n, cnt)
        total_time += time.perf_counter() - t0
        total_flops += n ** 3 / 3.0 * cnt
        parts.append(f"dpotrf n={n}: {cnt} instances")
    # one host thread on a smaller sample (1/16 of the flops per case)
    one_flops, one_time = 0.0, 0.0
    for (n, batch, A, B, C) in gemm:
        cnt = int(max(1, min(batch, flops_per_case / 16 // (2 * n ** 3))))
        a = A[:cnt].transpose(1, 2).contiguous().cpu().numpy().ravel()
        b = B[:cnt].transpose(1, 2).contiguous().cpu().numpy().ravel()
        c = C[:cnt].transpose(1, 2).contiguous().cpu().numpy().ravel()
        t0 = time.perf_counter()
        oracle.dgemm_strided_batched("N", "N", n, n, n, 1.0, a, n, n * n, b, n, n * n, 1.0, c, n,
                                     n * n, cnt, nthreads=1)
        one_time += time.perf_counter() - t0
        one_flops += 2.0 * n ** 3 * cnt
    return {
        "value": total_flops / total_time / 1e9,
        "unit": "GFLOP/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "seconds": round(total_time, 2),
        "sample": "leading instances of every sweep case, about "
                  f"{flops_per_case / 1e9:.1f} GFLOP per case: " + "; ".join(parts),
        "value_1_thread": round(one_flops / one_time / 1e9, 3),
        "sample_1_thread": "dgemm NN, leading instances of every sweep size, about "
                           f"{flops_per_case / 16 / 1e9:.2f} GFLOP per size",
        "cpu_model": host_cpu_model(),
    }


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def single_call(torch, _lib, oracle, inputs):
    """The single plain call: dgemm NN, m = n = k = 32, lda = 32, alpha = beta =
    1, U[-1,1) from the seed scheme; parity against the oracle and the call's
    latency (HIP events around each call, median and min of 100)."""
    n = 32
    g = inputs.rng(inputs.seed_for(0, 0))
    A = inputs.colmajor(g, 1, n, n)
    B = inputs.colmajor(g, 1, n, n)
    C = inputs.colmajor(g, 1, n, n)
    dA, dB = (torch.from_numpy(X.ravel().copy()).cuda() for X in (A, B))
    dC = torch.from_numpy(C.ravel().copy()).cuda()
    st = _lib.dgemm("N", "N", n, n, n, 1.0, dA.data_ptr(), n, dB.data_ptr(), n, 1.0, dC.data_ptr(),
                    n, torch.cuda.current_stream().cuda_stream)
    assert st == 0, st
    torch.cuda.synchronize()
    ref = C.ravel().copy()
    oracle.dgemm_raw("N", "N", n, n, n, 1.0, A.ravel().copy(), n, B.ravel().copy(), n, 1.0, ref, n)
    got = dC.cpu().numpy()
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    work = torch.from_numpy(C.ravel().copy()).cuda()

    def call():
        _lib.dgemm("N", "N", n, n, n, 1.0, dA.data_ptr(), n, dB.data_ptr(), n, 1.0,
                   work.data_ptr(), n, torch.cuda.current_stream().cuda_stream)
    for _ in range(10):
        call()
    ts = []
    for _ in range(100):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        call()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3)
    return {"m": n, "n": n, "k": n, "kernel": _lib.dgemm_kernel_name("N", "N", n, n, n),
            "rel_err": err, "pass": err <= 1e-12, "latency_us_median": round(float(np.median(ts)), 2),
            "latency_us_min": round(float(min(ts)), 2)}


def parity_spot_check(torch, _lib, oracle, gemm, potrf, stream):
    """Untimed: one more call per case on sampled instances vs the oracle."""
    sh = stream.cuda_stream
    worst_gemm = 0.0
    for (n, batch, A, B, C) in gemm:
        if n not in (4, 12, 64, 192, 300):
            continue
        idx = torch.tensor([0, batch // 2, batch - 1], device="cuda")
        for trans in ("NN", "NT", "TN", "TT"):
            a0 = A[idx].cpu().numpy()
            b0 = B[idx].cpu().numpy()
            c0 = C[idx].cpu().numpy()
            st = _lib.dgemm_strided_batched(trans[0], trans[1], n, n, n, 1.0, A.data_ptr(), n,
                                            n * n, B.data_ptr(), n, n * n, 1.0, C.data_ptr(), n,
                                            n * n, batch, sh)
            assert st == 0
            cg = C[idx].cpu().numpy()
            for j in range(3):
                cr = np.asfortranarray(c0[j].copy())
                oracle.dgemm(trans[0], trans[1], 1.0, np.asfortranarray(a0[j]),
                             np.asfortranarray(b0[j]), 1.0, cr)
                worst_gemm = max(worst_gemm, np.linalg.norm(cg[j] - cr) / np.linalg.norm(cr))
    worst_res = 0.0
    info_ok = True
    for (n, batch, master, copies, info, (bad_b, bad_j)) in potrf:
        X = master.clone()
        st = _lib.dpotrf_strided_batched("L", n, X.data_ptr(), n, n * n, info.data_ptr(), batch,
                                         sh)
        assert st == 0
        inf = info.cpu().numpy()
        exp = np.zeros(batch, dtype=np.int32)
        exp[bad_b] = bad_j + 1
        info_ok = info_ok and bool(np.array_equal(inf, exp))
        for b in (0, batch - 1):
            if b == bad_b:
                continue
            a0 = master[b].cpu().numpy().astype(np.longdouble)
            lg = np.tril(X[b].cpu().numpy()).astype(np.longdouble)
            r = np.sqrt(((a0 - lg @ lg.T) ** 2).sum() / (a0 ** 2).sum())
            worst_res = max(worst_res, float(r))
        del X
    return {"dgemm_max_rel_err": float(worst_gemm), "dpotrf_max_residual": float(worst_res),
            "dpotrf_info_exact": info_ok, "tolerance": 1e-12,
            "pass": bool(worst_gemm <= 1e-12 and worst_res <= 1e-12 and info_ok)}


def crossover(torch, _lib, inputs, args):
    """The size switch measured: the direct, packed and register-tile kernel
    families (and the automatic choice) at every sweep size and trans case."""
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    rows = []
    for n in args.gemm_sizes:
        batch = inputs.gemm_sweep_batch(n)
        A = inputs.torch_colmajor(batch, n, n, seed=1)
        B = inputs.torch_colmajor(batch, n, n, seed=2)
        C = inputs.torch_colmajor(batch, n, n, seed=3)
        for trans in ("NN", "NT", "TN", "TT"):
            res = {}
            for vname, v in (("direct", 1), ("packed", 2), ("regtile", 3), ("auto", 0)):
                def call():
                    st = _lib.dgemm_strided_batched(trans[0], trans[1], n, n, n, 1.0,
                                                    A.data_ptr(), n, n * n, B.data_ptr(), n,
                                                    n * n, 1.0, C.data_ptr(), n, n * n, batch,
                                                    sh, v)
                    assert st == 0
                for _ in range(2):
                    call()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(args.steps):
                    call()
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / args.steps
                fl, by = gemm_work(n, batch)
                res[vname] = {"ms": ms, "gflops": fl / ms / 1e6, "gbps": by / ms / 1e6,
                              "kernel": _lib.dgemm_kernel_name(trans[0], trans[1], n, n, n, v)}
            fam = {k: v for k, v in res.items() if k != "auto"}
            rows.append({"n": n, "trans": trans, "batch": batch, **res,
                         "faster": min(fam, key=lambda k: fam[k]["ms"])})
            log(f"crossover n={n} {trans}: " + ", ".join(
                f"{k} {v['gflops']:.0f} GF/s" for k, v in res.items()))
        del A, B, C
        torch.cuda.empty_cache()
    print(json.dumps({"crossover": rows}))


def time_events(torch, fn, reps, setup=None):
    """Best and median of `reps` timed calls of fn (events on the current
    stream); setup() runs untimed before each call."""
    ts = []
    for _ in range(reps):
        if setup is not None:
            setup()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return min(ts), float(np.median(ts))


def uneven_batch(torch, _lib, inputs, reps, modes=("fused_graph", "fused", "grouped_graph",
                                                   "grouped")):
    """The uneven batch (100,000 problems, sizes log-uniform 4..160, 70% dgemm
    / 30% dpotrf) through one plan: the fused persistent kernel (graph and
    direct launch) against per-shape grouped batched calls (raw and
    graph-captured).  Inputs are restored (untimed) before every execution,
    since dpotrf works in place."""
    from paper_1902_08115_amd import blas
    spec = inputs.uneven_spec(inputs.UNEVEN_COUNT, inputs.seed_for(3, 0))
    X0 = inputs.uneven_device(spec, inputs.seed_for(3, 200))
    X = X0.clone()
    info = torch.zeros(spec["count"], dtype=torch.int32, device="cuda")
    base, ib = X.data_ptr(), info.data_ptr()
    probs = []
    for i in range(spec["count"]):
        if spec["op"][i] == 0:
            probs.append(dict(op=0, transa="NT"[spec["ta"][i]], transb="NT"[spec["tb"][i]],
                              m=spec["m"][i], n=spec["n"][i], k=spec["k"][i], lda=spec["lda"][i],
                              ldb=spec["ldb"][i], ldc=spec["ldc"][i], alpha=1.0, beta=1.0,
                              A=base + 8 * int(spec["off_a"][i]),
                              B=base + 8 * int(spec["off_b"][i]),
                              C=base + 8 * int(spec["off_c"][i])))
        else:
            probs.append(dict(op=1, uplo="L", n=spec["n"][i], ldc=spec["ldc"][i],
                              C=base + 8 * int(spec["off_c"][i]), info=ib + 4 * i))
    t0 = time.perf_counter()
    plan = blas.Plan(probs)
    create_s = time.perf_counter() - t0
    st = plan.stats()
    g = spec["op"] == 0
    m, n, k = spec["m"], spec["n"], spec["k"]
    flops = float((2.0 * m * n * k)[g].sum() + (n[~g].astype(float) ** 3 / 3).sum())
    nbytes = float(((m * k + k * n + 2 * m * n) * 8)[g].sum()
                   + (n[~g] * (n[~g] + 1) * 8).astype(float).sum())
    restore = lambda: X.copy_(X0)  # noqa: E731
    res = {}
    for mode in modes:
        r = reps if mode.startswith("fused") else 2
        md = getattr(blas.Plan, mode.upper())
        restore()
        plan.execute(md)  # warm (captures the grouped graph on first use)
        torch.cuda.synchronize()
        best, med = time_events(torch, lambda: plan.execute(md), r, restore)
        res[mode] = {"best_ms": round(best, 4), "median_ms": round(med, 4),
                     "gflops": round(flops / best / 1e6, 1)}
        log(f"uneven batch {mode}: {best:.3f} ms ({flops / best / 1e6:.0f} GFLOP/s)")
    plan.close()
    fb = res["fused_graph" if "fused_graph" in res else modes[0]]["best_ms"]
    grouped = {k: round(res[k]["best_ms"] / fb, 1) for k in ("grouped", "grouped_graph")
               if k in res}
    return {
        "workload": "uneven batch: %d problems, sizes floor(exp(U[ln 4, ln 161))), 70%% dgemm "
                    "(m, n, k independent, transa/transb uniform, alpha = beta = 1) / 30%% "
                    "dpotrf L (SPD), tight ld, one arena" % spec["count"],
        "flops": flops, "algorithmic_bytes": nbytes,
        "fused_gbps": round(nbytes / fb / 1e6, 1),
        "fused_traffic_bytes": traffic_for("fused_kernel", nbytes),
        "hbm_roofline_ms": round(nbytes / (PEAK_HBM_GBS * 1e9) * 1e3, 4),
        "modes": res,
        "speedup_vs": grouped,
        "plan": {k2: int(v) for k2, v in st.items()}, "plan_create_s": round(create_s, 3),
    }


def skinny_sweeps(torch, _lib, inputs, reps):
    """The paper's rectangular sweeps (App. C): m = n = 4 with k = s, m = 4
    with n = k = s, n = 4 with m = k = s, s over the square sweep sizes, every
    trans case, through the shape-aware dispatch; batch for ~1 GiB of
    operands per point (beyond the 256 MiB last-level cache).  Reports the
    kernel chosen and GFLOP/s and GB/s."""
    sh = torch.cuda.current_stream().cuda_stream
    out = []
    for label, shape in (("m=n=4", lambda s: (4, 4, s)), ("m=4", lambda s: (4, s, s)),
                         ("n=4", lambda s: (s, 4, s))):
        for s in inputs.GEMM_SWEEP_SIZES:
            m, n, k = shape(s)
            for t in inputs.TRANS_CASES:
                ar, ac = (m, k) if t[0] == "N" else (k, m)
                br, bc = (k, n) if t[1] == "N" else (n, k)
                batch = min(1 << 22, (1 << 30) // (8 * (m * k + k * n + m * n)))
                A = inputs.torch_colmajor(batch, ar, ac, seed=21)
                B = inputs.torch_colmajor(batch, br, bc, seed=22)
                C = inputs.torch_colmajor(batch, m, n, seed=23)
                fn = lambda: _lib.dgemm_strided_batched(  # noqa: E731
                    t[0], t[1], m, n, k, 1.0, A.data_ptr(), ar, ar * ac, B.data_ptr(), br,
                    br * bc, 1.0, C.data_ptr(), m, m * n, batch, sh)
                fn()
                best, _ = time_events(torch, fn, reps)
                fl = 2.0 * m * n * k * batch
                by = 8.0 * (m * k + k * n + 2 * m * n) * batch
                out.append({"sweep": label, "m": m, "n": n, "k": k, "trans": t, "batch": batch,
                            "kernel": _lib.dgemm_kernel_name(t[0], t[1], m, n, k),
                            "ms": round(best, 4), "gflops": round(fl / best / 1e6, 1),
                            "gbps": round(by / best / 1e6, 1)})
                del A, B, C
            log(f"skinny {label} s={s}: " + " ".join(
                f"{r['trans']} {r['gbps']:.0f}GB/s" for r in out[-4:]))
    torch.cuda.empty_cache()
    return out


def backward_workload(torch, _lib, inputs, reps):
    """The differentiation workload: C = chol(A) B (B n x 32) forward and
    backward through the autograd Functions for 8192 instances of order 64,
    and through fused plans for 2048 instances of orders 16..192."""
    from paper_1902_08115_amd import autograd as ag
    from paper_1902_08115_amd.mixed import MixedCholeskyProduct
    out = {}
    batch, n, nb = inputs.BACKWARD_BATCH, inputs.BACKWARD_N, inputs.BACKWARD_NB
    A = inputs.torch_spd(batch, n, seed=inputs.seed_for(4, 1))
    B = inputs.torch_colmajor(batch, n, nb, seed=inputs.seed_for(4, 2))
    W = inputs.torch_colmajor(batch, n, nb, seed=inputs.seed_for(4, 3))
    Ar, Br = A.detach().requires_grad_(True), B.detach().requires_grad_(True)
    state = {}

    def fwd():
        state["C"] = ag.cholesky_product(Ar, Br)

    def bwd():
        state["C"].backward(W)

    def fresh():  # a new graph and no accumulated gradients before each timed backward
        Ar.grad = None
        Br.grad = None
        fwd()

    fwd()
    bwd()
    torch.cuda.synchronize()
    f_best, _ = time_events(torch, fwd, reps)
    b_best, _ = time_events(torch, bwd, reps, fresh)
    ffl = batch * (n ** 3 / 3 + 2.0 * n * n * nb)
    bfl = batch * (4.0 * n * n * nb + 5.0 * n ** 3 / 3)
    out["n64_batch8192"] = {"forward_ms": round(f_best, 4), "backward_ms": round(b_best, 4),
                            "forward_gflops": round(ffl / f_best / 1e6, 1),
                            "backward_gflops": round(bfl / b_best / 1e6, 1)}
    log(f"backward n=64 x 8192: forward {f_best:.3f} ms, backward {b_best:.3f} ms")
    # the Cholesky adjoint kernel alone (one launch over the 8192 instances):
    # P = Phi(L^T Lbar) and the two triangular solves, about 5 n^3 / 3 flop;
    # L and Lbar lower triangles read, Abar written whole
    Lt = ag.cholesky(A.detach())
    Lbar = torch.tril(inputs.torch_colmajor(batch, n, n, seed=inputs.seed_for(4, 5)))
    Lbar = ag.colmajor(Lbar)
    Abar = torch.empty_like(Lbar)
    sh = torch.cuda.current_stream().cuda_stream

    def adj():
        st = _lib.dpotrf_l_backward_strided_batched(n, Lt.data_ptr(), n, n * n, Lbar.data_ptr(),
                                                    n, n * n, Abar.data_ptr(), n, n * n, batch, sh)
        assert st == 0, st
    adj()
    a_best, a_med = time_events(torch, adj, reps)
    afl = batch * 5.0 * n ** 3 / 3
    aby = batch * (8.0 * n * (n + 1) + 8.0 * n * n)
    roof = min(PEAK_FP64_TFLOPS, afl / aby * PEAK_HBM_GBS / 1e3)
    out["adjoint_kernel_n64_batch8192"] = {
        "kernel": "potrf_adj_regs_kernel<4>", "ms": round(a_best, 4), "median_ms": round(a_med, 4),
        "flops": afl, "algorithmic_bytes": aby, "gflops": round(afl / a_best / 1e6, 1),
        "gbps": round(aby / a_best / 1e6, 1), "roofline_tflops": round(roof, 2),
        "roof_frac": round(afl / a_best / 1e9 / roof, 3)}
    log(f"cholesky adjoint kernel n=64 x 8192: {a_best:.3f} ms "
        f"({out['adjoint_kernel_n64_batch8192']['roof_frac']} of its roofline)")
    del Lt, Lbar, Abar
    ns = inputs.backward_mixed_sizes(inputs.seed_for(4, 10))
    mp = MixedCholeskyProduct(ns, nb)
    for v in np.unique(ns):
        idx = np.nonzero(ns == v)[0]
        S = inputs.torch_spd(len(idx), int(v), seed=inputs.seed_for(4, 20000 + int(v)))
        for j, b in enumerate(idx):
            mp.view("A", int(b)).copy_(S[j])
    gen = torch.Generator(device="cuda")
    mp.buf["B"].uniform_(-1.0, 1.0, generator=gen.manual_seed(12))
    Wm = torch.empty_like(mp.buf["C"]).uniform_(-1.0, 1.0, generator=gen.manual_seed(13))
    # through the autograd Function, on the object's own arenas (no input copies)
    Am = mp.buf["A"].requires_grad_(True)
    Bm = mp.buf["B"].requires_grad_(True)

    def mfwd():
        state["Cm"] = mp(Am, Bm)

    def mbwd():
        state["Cm"].backward(Wm)

    def mfresh():
        Am.grad = None
        Bm.grad = None
        mfwd()

    mfwd()
    mbwd()
    torch.cuda.synchronize()
    f_best, _ = time_events(torch, mfwd, reps)
    b_best, _ = time_events(torch, mbwd, reps, mfresh)
    nf = ns.astype(float)
    ffl = float((nf ** 3 / 3 + 2.0 * nf * nf * nb).sum())
    bfl = float((4.0 * nf * nf * nb + 5.0 * nf ** 3 / 3).sum())
    out["mixed_2048_n16_192"] = {"forward_ms": round(f_best, 4), "backward_ms": round(b_best, 4),
                                 "forward_gflops": round(ffl / f_best / 1e6, 1),
                                 "backward_gflops": round(bfl / b_best / 1e6, 1)}
    log(f"backward mixed 2048: forward {f_best:.3f} ms, backward {b_best:.3f} ms")
    mp.close()
    return out


def riccati_flops(nx, nu, N):
    """Flops of one recursion by the paper's counting (App. D, Table 3: dsyrk
    n^3, dpotrf n^3/3 for n x n operands; dtrmm of an m x n by an n x n
    triangle m n^2): per stage m nx^2 + m^2 nx + m^3/3, plus nx^3/3."""
    m = nu + nx
    return N * (m * nx * nx + m * m * nx + m ** 3 / 3.0) + nx ** 3 / 3.0


def riccati_bytes(nx, nu, N):
    """Algorithmic HBM bytes of one recursion: BAt_n read, lower triangles of
    RSQ_n and Q_N read, lower triangles of F_n and LN written, once each."""
    m = nu + nx
    tri_m, tri_x = m * (m + 1) // 2, nx * (nx + 1) // 2
    return 8.0 * (N * (m * nx + 2 * tri_m) + 2 * tri_x)


# Table 2 of the paper, BLASFEO API from C on one Haswell core at 3.4 GHz:
# seconds per recursion (N = 10) -- context only, another machine and one
# problem at a time.
PAPER_RICCATI_S = {(8, 4): 3.24e-6, (24, 12): 2.29e-5, (40, 20): 7.95e-5, (64, 32): 2.87e-4}


def riccati_workload(torch, _lib, inputs, reps, composed=True):
    """The Riccati recursion of Sec. 5.2 at the paper's four (nx, nu), N = 10,
    batched over independent problems: the fused one-wave-per-problem kernel,
    and (composed) the same recursion as 3 N + 1 batched library calls --
    dtrmm_rlnn, dsyrk_ln, dpotrf per stage, the routines the paper names --
    in place on copies of the inputs (made outside the timed region)."""
    from paper_1902_08115_amd import blas
    out = {}
    N = inputs.RICCATI_N
    stream = torch.cuda.current_stream()
    for (nx, nu) in inputs.RICCATI_SHAPES:
        m = nx + nu
        batch = inputs.RICCATI_BATCH[(nx, nu)]
        BAt, RSQ, QN = inputs.torch_riccati(nx, nu, N, batch, inputs.seed_for(42, nx))
        F = torch.zeros((batch, N, m, m), dtype=torch.float64, device="cuda").transpose(2, 3)
        LN = torch.zeros((batch, nx, nx), dtype=torch.float64, device="cuda").transpose(1, 2)
        info = torch.empty((batch, N + 1), dtype=torch.int32, device="cuda")
        work = blas.riccati_workspace(nx, nu, batch)

        def fused():
            blas.riccati(BAt, RSQ, QN, nu, F=F, LN=LN, info=info, work=work, stream=stream)

        fused()
        torch.cuda.synchronize()
        assert int((info != 0).sum()) == 0, "Riccati factorization failed on SPD inputs"
        best, med = time_events(torch, fused, reps)
        fl, by = riccati_flops(nx, nu, N) * batch, riccati_bytes(nx, nu, N) * batch
        rec = {"batch": batch, "N": N, "ms": round(best, 4), "median_ms": round(med, 4),
               "recursions_per_s": round(batch / best * 1e3, 1),
               "us_per_recursion_amortized": round(best * 1e3 / batch, 5),
               "gflops": round(fl / best / 1e6, 1), "gbps": round(by / best / 1e6, 1),
               "roof_frac": round((fl / best / 1e9) / min(PEAK_FP64_TFLOPS,
                                                          fl / by * PEAK_HBM_GBS / 1e3), 3),
               "kernel": riccati_kernel_label(nx, nu),
               "flops_per_recursion": riccati_flops(nx, nu, N),
               "bytes_per_recursion": riccati_bytes(nx, nu, N),
               "paper_blasfeo_api_c_haswell_s_per_recursion": PAPER_RICCATI_S[(nx, nu)]}
        log(f"riccati nx={nx} nu={nu} N={N} batch={batch}: fused {best:.3f} ms "
            f"({rec['gflops']} GFLOP/s, {rec['gbps']} GB/s)")
        if composed:
            Fc = RSQ.clone()
            Lc = QN.clone()
            Cc = BAt.clone()
            infc = torch.empty((batch,), dtype=torch.int32, device="cuda")
            s = stream.cuda_stream
            ldf, stf, sf = m, m * m, N * m * m
            ldb, stb, sb = m, m * nx, N * m * nx

            def reset():
                Fc.copy_(RSQ)
                Lc.copy_(QN)
                Cc.copy_(BAt)

            def comp():
                st = _lib.dpotrf_strided_batched("L", nx, Lc.data_ptr(), nx, nx * nx,
                                                 infc.data_ptr(), batch, s)
                assert st == 0
                prev, ldp, sp = Lc.data_ptr(), nx, nx * nx
                for n in range(N - 1, -1, -1):
                    fb = Fc.data_ptr() + 8 * n * stf
                    cb = Cc.data_ptr() + 8 * n * stb
                    st = _lib.dtrmm_rlnn_strided_batched(m, nx, 1.0, prev, ldp, sp, cb, ldb, sb,
                                                         batch, s)
                    assert st == 0
                    st = _lib.dsyrk_ln_strided_batched(m, nx, 1.0, cb, ldb, sb, 1.0, fb, ldf, sf,
                                                       batch, s)
                    assert st == 0
                    st = _lib.dpotrf_strided_batched("L", m, fb, ldf, sf, infc.data_ptr(), batch, s)
                    assert st == 0
                    prev, ldp, sp = fb + 8 * (nu + nu * ldf), ldf, sf

            reset()
            comp()
            torch.cuda.synchronize()
            d = float((torch.tril(Fc) - torch.tril(F)).abs().max() / torch.tril(F).abs().max())
            cbest, cmed = time_events(torch, comp, reps, reset)
            rec["composed"] = {"ms": round(cbest, 4), "median_ms": round(cmed, 4),
                               "launches": 3 * N + 1, "speedup_fused": round(cbest / best, 2),
                               "max_rel_diff_vs_fused": d}
            log(f"  composed 3N+1 launches: {cbest:.3f} ms (fused x{cbest / best:.2f}), "
                f"diff {d:.1e}")
            del Fc, Lc, Cc
        out[f"nx{nx}_nu{nu}"] = rec
        del BAt, RSQ, QN, F, LN, work
        torch.cuda.empty_cache()
    return out


def compact_line(head, args, restore_bytes, peak_frac, roofline, cpu, per_size, ceil, parity,
                 single, nxt, potrf_top=None):
    """The one stdout line: the headline, the dominant kernel's roofline (and
    the largest dpotrf order's, which led the kernel time before), the CPU
    baseline and GFLOP/s against n per routine (best trans case for dgemm),
    kept short enough to be read whole (about 1.7 KB)."""
    def best_gemm(n):
        return max(per_size[f"dgemm_{t}_n{n}"]["gflops"] for t in ("NN", "NT", "TN", "TT"))
    out = dict(head)
    out["config"] = {"workload": "dgemm sweep n=%s x4 trans (~1 GiB each) + dpotrf L n=%s x %d"
                                 % (",".join(map(str, args.gemm_sizes)),
                                    ",".join(map(str, args.potrf_sizes)), args.potrf_batch),
                     "potrf_input_copies": args.copies,
                     "restore_bytes_per_step": restore_bytes}
    out["fp64_peak_frac"] = peak_frac
    out["roofline"] = {k: roofline[k] for k in ("bound", "achieved", "peak", "unit", "frac",
                                                "traffic", "kernel", "avg_launch_ms")}
    if potrf_top is not None and potrf_top["kernel"] != roofline["kernel"]:
        out["roofline_dpotrf_largest"] = {k: potrf_top[k] for k in (
            "kernel", "bound", "achieved", "unit", "frac", "traffic", "avg_launch_ms")}
    if cpu is not None:
        out["cpu_baseline"] = {"value": round(cpu["value"], 2), "unit": cpu["unit"],
                               "cores": cpu["cores"], "kind": "oracle",
                               "sample": "leading instances of every sweep case, %.0f GFLOP "
                                         "per case, %.1f s" % (args.cpu_flops_per_case / 1e9,
                                                               cpu["seconds"]),
                               "value_1_thread": cpu["value_1_thread"],
                               "cpu_model": cpu["cpu_model"]}
    out["gflops_vs_n"] = {
        "dgemm_best_trans": {str(n): best_gemm(n) for n in args.gemm_sizes},
        "dpotrf": {str(n): per_size[f"dpotrf_n{n}"]["gflops"] for n in args.potrf_sizes}}
    out["hbm_ceiling_gbps"] = {k: ceil.get(k) for k in ("hbm_read_gbps", "hbm_copy_gbps",
                                                        "hbm_3r1w_gbps")}
    if parity is not None:
        out["parity"] = {"pass": parity["pass"], "dgemm_max_rel_err": parity["dgemm_max_rel_err"],
                         "dpotrf_max_residual": parity["dpotrf_max_residual"],
                         "info_exact": parity["dpotrf_info_exact"]}
    if single is not None:
        out["single_call"] = {"kernel": single["kernel"], "rel_err": single["rel_err"],
                              "latency_us_median": single["latency_us_median"]}
    if nxt is not None:
        ub = nxt["uneven_batch"]
        out["fused_vs_plain"] = {"fused_graph_ms": ub["modes"]["fused_graph"]["best_ms"],
                                 "speedup": ub["speedup_vs"]}
    return json.dumps(out, separators=(",", ":"))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--copies", type=int, default=None,
                    help="pristine dpotrf input copies (default: one per timed step, as many as "
                         "device memory holds)")
    ap.add_argument("--details-out", type=str, default=None,
                    help="also write the full per-size / per-kernel record to this JSON file")
    ap.add_argument("--gemm-sizes", type=str, default=None)
    ap.add_argument("--potrf-sizes", type=str, default=None)
    ap.add_argument("--potrf-batch", type=int, default=None)
    ap.add_argument("--cpu-flops-per-case", type=float, default=2.0e10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--crossover", action="store_true")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the uneven-batch and differentiation measurements")
    ap.add_argument("--next-only", action="store_true",
                    help="only the uneven-batch and differentiation measurements (profiling)")
    ap.add_argument("--skinny", action="store_true",
                    help="also measure the thin / flat / small dgemm sweeps")
    ap.add_argument("--uneven-modes", type=str, default="fused_graph,fused,grouped_graph,grouped",
                    help="plan execution modes timed on the uneven batch")
    ap.add_argument("--riccati-only", action="store_true",
                    help="only the Riccati recursion workload (profiling)")
    ap.add_argument("--next-parts", type=str, default="uneven,backward,riccati",
                    help="with --next-only: which of the uneven batch, differentiation and "
                         "Riccati workloads run (profiling one workload at a time)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (--gpus {args.gpus} requested); the "
              "batched path shards by splitting the batch across GPUs with no exchange, which "
              "is not run here.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1902_08115_amd import _lib, inputs
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")

    def sizes(text, default):
        if not text:
            return list(default)
        if text == "none":
            return []
        return [int(x) for x in text.split(",")]
    args.gemm_sizes = sizes(args.gemm_sizes, inputs.GEMM_SWEEP_SIZES)
    args.potrf_sizes = sizes(args.potrf_sizes, inputs.POTRF_SWEEP_SIZES)
    args.potrf_batch = args.potrf_batch or inputs.POTRF_SWEEP_BATCH
    if args.copies is None:
        # one factored copy per timed step, so that no timed step restores its
        # input; bounded by what the device holds next to the dgemm operands
        per_copy = sum(8 * n * n * args.potrf_batch for n in args.potrf_sizes) or 1
        gemm_bytes = sum(3 * 8 * n * n * inputs.gemm_sweep_batch(n) for n in args.gemm_sizes)
        total = torch.cuda.get_device_properties(0).total_memory
        room = total - gemm_bytes - per_copy - (24 << 30)
        args.copies = max(1, min(args.steps, room // per_copy))

    # no garbage collection while anything is timed (as timeit does): a full
    # collection over the interpreter's objects stalls the submitting thread
    # long enough to drain the launch queue; nothing here depends on cycles
    # being freed
    gc.collect()
    gc.disable()

    if args.crossover:
        crossover(torch, _lib, inputs, args)
        return
    if args.riccati_only:
        print(json.dumps({"next": {"riccati": riccati_workload(torch, _lib, inputs, args.steps)}}),
              flush=True)
        return
    if args.next_only:
        parts = args.next_parts.split(",")
        nxt = {}
        if "uneven" in parts:
            nxt["uneven_batch"] = uneven_batch(torch, _lib, inputs, args.steps,
                                               args.uneven_modes.split(","))
        if "backward" in parts:
            nxt["backward"] = backward_workload(torch, _lib, inputs, args.steps)
        if "riccati" in parts:
            nxt["riccati"] = riccati_workload(torch, _lib, inputs, args.steps)
        if args.skinny:
            nxt["skinny"] = skinny_sweeps(torch, _lib, inputs, args.steps)
        print(json.dumps({"next": nxt}), flush=True)
        return

    log(f"device {torch.cuda.get_device_name(0)}; generating inputs")
    gemm, potrf = build_inputs(torch, inputs, args)
    log("inputs resident")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(torch, oracle, gemm, potrf, args.cpu_flops_per_case)
        log(f"cpu baseline {cpu['value']:.2f} GFLOP/s on {cpu['cores']} threads "
            f"({cpu['seconds']} s)")

    stream = torch.cuda.current_stream()
    restore = [0]
    for w in range(args.warmup):
        run_step(w, gemm, potrf, _lib, stream, None, restore)
    # the copies the warmup factored are restored here, outside the timed steps
    for (n, batch, master, copies, info, _) in potrf:
        for c in copies[:min(args.warmup, len(copies))]:
            c.copy_(master)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    timer = Timer(torch)
    restore = [0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        run_step(s, gemm, potrf, _lib, stream, timer, restore)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step")
    durations = timer.collect()

    # the same dpotrf sizes with a hot input, and the measured ceilings
    # (both outside the timed steps)
    hot = potrf_hot(torch, _lib, potrf, stream)
    ceil = ceilings(torch, _lib, stream)
    log(f"ceilings: {ceil}")

    # per-call and per-kernel-class accounting
    per_size = {}
    classes = {}
    step_flops = 0.0
    for (n, batch, *_r) in gemm:
        fl, by = gemm_work(n, batch)
        for trans in ("NN", "NT", "TN", "TT"):
            ds = durations[("dgemm", trans, n)]
            ms = float(np.median(ds))
            kname = f"{_lib.dgemm_kernel_name(trans[0], trans[1], n, n, n)}_{trans}"
            per_size[f"dgemm_{trans}_n{n}"] = {
                "kernel": kname, "batch": batch, "ms": round(ms, 4), "ms_min": round(min(ds), 4),
                "gflops": round(fl / ms / 1e6, 1), "gbps": round(by / ms / 1e6, 1),
                "roof_frac": round((fl / ms / 1e9) / min(PEAK_FP64_TFLOPS,
                                                          fl / by * PEAK_HBM_GBS / 1e3), 3)}
            c = classes.setdefault(kname, {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
            cnt = len(ds)
            c["ms"] += float(np.sum(ds))
            c["launches"] += cnt
            c["flops"] += fl * cnt
            c["bytes"] += by * cnt
            step_flops += fl
    for (n, batch, *_r) in potrf:
        fl, by = potrf_work(n, batch)
        ds = durations[("dpotrf", "L", n)]
        ms = float(np.median(ds))
        kname = _lib.dpotrf_kernel_name(n)
        per_size[f"dpotrf_n{n}"] = {
            "kernel": kname, "batch": batch, "ms": round(ms, 4), "ms_min": round(min(ds), 4),
            "gflops": round(fl / ms / 1e6, 1), "gbps": round(by / ms / 1e6, 1),
            # LAPACK's exact count n^3/3 + n^2/2 + n/6 instead of the paper's n^3/3
            "gflops_lapack_count": round((n ** 3 / 3 + n ** 2 / 2 + n / 6) * batch / ms / 1e6, 1),
            # "ms" above is cold (the step's rotating input copies); "hot" restores
            # the input right before each timed factorization
            "hot": hot[n],
            "roof_frac": round((fl / ms / 1e9) / min(PEAK_FP64_TFLOPS,
                                                      fl / by * PEAK_HBM_GBS / 1e3), 3)}
        c = classes.setdefault(kname, {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
        cnt = len(ds)
        c["ms"] += float(np.sum(ds))
        c["launches"] += cnt
        c["flops"] += fl * cnt
        c["bytes"] += by * cnt
        step_flops += fl

    kernels = {}
    for k, c in classes.items():
        ai = c["flops"] / c["bytes"]
        bound = "mfma" if ai >= RIDGE else "hbm"
        avg_ms = c["ms"] / c["launches"]
        if bound == "mfma":
            ach = c["flops"] / (c["ms"] * 1e-3) / 1e12
            peak, unit = PEAK_FP64_TFLOPS, "TFLOP/s"
        else:
            ach = c["bytes"] / (c["ms"] * 1e-3) / 1e9
            peak, unit = PEAK_HBM_GBS, "GB/s"
        kernels[k] = {"bound": bound, "achieved": round(ach, 2), "peak": peak, "unit": unit,
                      "frac": round(ach / peak, 4), "avg_launch_ms": round(avg_ms, 4),
                      "launches_per_step": c["launches"] // args.steps,
                      "share_of_kernel_time": None, "flops_per_launch": c["flops"] / c["launches"],
                      "bytes_per_launch": c["bytes"] / c["launches"]}
    total_kernel_ms = sum(c["ms"] for c in classes.values())
    for k in kernels:
        kernels[k]["share_of_kernel_time"] = round(classes[k]["ms"] / total_kernel_ms, 4)
    dom = max(kernels, key=lambda k: classes[k]["ms"])
    d = kernels[dom]
    roofline = {"kernel": dom, "bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"],
                "unit": d["unit"], "frac": d["frac"],
                "traffic": traffic_for(dom, d["bytes_per_launch"]),
                "algorithmic_bytes_per_launch": d["bytes_per_launch"],
                "algorithmic_flops_per_launch": d["flops_per_launch"],
                "avg_launch_ms": d["avg_launch_ms"]}
    potrf_top = None
    if args.potrf_sizes:
        pk = _lib.dpotrf_kernel_name(max(args.potrf_sizes))
        if pk in kernels:
            p = kernels[pk]
            potrf_top = {"kernel": pk, "bound": p["bound"], "achieved": p["achieved"],
                         "unit": p["unit"], "frac": p["frac"],
                         "traffic": traffic_for(pk, p["bytes_per_launch"]),
                         "avg_launch_ms": p["avg_launch_ms"]}

    parity = None
    single = None
    if not args.no_parity:
        import oracle
        log("parity spot check")
        parity = parity_spot_check(torch, _lib, oracle, gemm, potrf, stream)
        single = single_call(torch, _lib, oracle, inputs)
        log(f"single dgemm 32^3: {single['latency_us_median']} us median, err {single['rel_err']:.1e}")

    nxt = None
    if not args.no_next:
        log("uneven batch (fused plan vs grouped launches)")
        nxt = {"uneven_batch": uneven_batch(torch, _lib, inputs, 5, args.uneven_modes.split(","))}
        log("differentiation workload")
        nxt["backward"] = backward_workload(torch, _lib, inputs, 5)
        log("Riccati recursion workload")
        nxt["riccati"] = riccati_workload(torch, _lib, inputs, 5)
        if args.skinny:
            log("thin / flat / small dgemm sweeps")
            nxt["skinny"] = skinny_sweeps(torch, _lib, inputs, 5)

    value = step_flops / (ms_per_step * 1e-3) / 1e9
    workload = ("square batched dgemm sweep (n in %s, NN/NT/TN/TT, alpha=beta=1, lda=n, batch "
                "~1 GiB of A+B+C per size) + batched dpotrf L sweep (n in %s, batch %d, one "
                "non-SPD instance per size)" % (args.gemm_sizes, args.potrf_sizes, args.potrf_batch))
    head = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
    }
    details = dict(head)
    details.update({
        "config": {
            "workload": workload,
            "gemm_sizes": args.gemm_sizes, "potrf_sizes": args.potrf_sizes,
            "potrf_batch": args.potrf_batch, "potrf_input_copies": args.copies,
            "restore_bytes_per_step": restore[0] / args.steps,
            "flops_per_step": step_flops,
        },
        "fp64_peak_frac": round(value / (PEAK_FP64_TFLOPS * 1e3), 4),
        "roofline": roofline,
        "roofline_dpotrf_largest": potrf_top,
        "ceilings": ceil,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "per_size": per_size,
        "parity": parity,
        "single_call": single,
        "next": nxt,
    })
    blob = json.dumps(details)
    if args.details_out:
        with open(args.details_out, "w") as f:
            f.write(blob + "\n")
    print(f"[bench] details {blob}", file=sys.stderr, flush=True)

    line = compact_line(head, args, restore[0] / args.steps, details["fp64_peak_frac"], roofline,
                        cpu, per_size, ceil, parity, single, nxt, potrf_top)
    print(line, flush=True)


if __name__ == "__main__":
    main()
