"""The benchmark's accounting on the CPU: the flop counts it divides by are the
paper's (App. D, Table 3, in tests/golden/flops.txt), its algorithmic bytes
are the operands read and written once, and its stdout record is one short
JSON line carrying the fields the measurement protocol names."""
import argparse
import json
import os

import bench

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "flops.txt")


def _table():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, expr = line.split()
        out[name] = expr
    return out


def test_flop_counts_follow_the_paper_table():
    tab = _table()
    for n in (4, 8, 37, 64, 300):
        for t in ("nn", "nt", "tn", "tt"):
            assert bench.gemm_work(n, 5)[0] == eval(tab[f"dgemm_{t}"], {"n": n}) * 5
        assert abs(bench.potrf_work(n, 3)[0] - eval(tab["dpotrf_l"], {"n": n}) * 3) <= 1e-9 * n ** 3


def test_algorithmic_bytes():
    n, b = 48, 7
    assert bench.gemm_work(n, b)[1] == 8 * (n * n + n * n + 2 * n * n) * b  # A, B read; C read+written
    assert bench.potrf_work(n, b)[1] == (8 * n * (n + 1) + 4) * b  # lower triangle twice, info


def test_compact_line_is_short_and_complete():
    sizes = [4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 300]
    psizes = [8, 16, 32, 64, 128, 192, 256]
    args = argparse.Namespace(gemm_sizes=sizes, potrf_sizes=psizes, potrf_batch=4096, copies=20,
                              cpu_flops_per_case=2e10)
    per_size = {f"dgemm_{t}_n{n}": {"gflops": 12345.6} for n in sizes
                for t in ("NN", "NT", "TN", "TT")}
    per_size.update({f"dpotrf_n{n}": {"gflops": 23456.7} for n in psizes})
    head = {"metric": bench.METRIC, "value": 24567.8, "unit": "GFLOP/s", "n_gpus": 1,
            "steps": 20, "warmup": 5, "ms_per_step": 18.6543, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    roof = {"bound": "mfma", "achieved": 45.93, "peak": 78.6, "unit": "TFLOP/s", "frac": 0.5843,
            "traffic": 1467363519, "kernel": "gemm_packed_tile64_k16_db_TT",
            "avg_launch_ms": 0.4791}
    potrf_top = {"kernel": "potrf_nt16", "bound": "mfma", "achieved": 24.36, "unit": "TFLOP/s",
                 "frac": 0.3099, "traffic": 5340990465, "avg_launch_ms": 0.9402}
    cpu = {"value": 45.123456, "unit": "GFLOP/s", "cores": 128, "seconds": 12.345,
           "value_1_thread": 4.456, "cpu_model": "AMD EPYC 9575F 64-Core Processor"}
    ceil = {"hbm_read_gbps": 6123.4, "hbm_copy_gbps": 5432.1, "hbm_3r1w_gbps": 5678.9}
    parity = {"pass": True, "dgemm_max_rel_err": 1.234e-16, "dpotrf_max_residual": 2.345e-16,
              "dpotrf_info_exact": True}
    single = {"kernel": "gemm_regtile_t22", "rel_err": 2.1e-16, "latency_us_median": 10.12}
    nxt = {"uneven_batch": {"modes": {"fused_graph": {"best_ms": 1.5234}},
                            "speedup_vs": {"grouped": 270.1, "grouped_graph": 280.2}}}
    line = bench.compact_line(head, args, 0.0, 0.3125, roof, cpu, per_size, ceil, parity, single,
                              nxt, potrf_top)
    assert "\n" not in line and len(line) <= 2048, len(line)
    rec = json.loads(line)
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config"):
        assert key in rec, key
    assert "workload" in rec["config"]
    assert set(rec["roofline"]) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert rec["roofline_dpotrf_largest"]["kernel"] == "potrf_nt16"
    assert set(rec["cpu_baseline"]) >= {"value", "unit", "cores", "kind", "sample"}
    assert rec["cpu_baseline"]["kind"] == "oracle"
    assert len(rec["gflops_vs_n"]["dgemm_best_trans"]) == len(sizes)
