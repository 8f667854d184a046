"""Benchmark: exact (17,6) planted motif search, n = 20, m = 600, on one GPU.

Prints one JSON line. `value` is Hamming tests per second: the canonical
number of Hamming tests of the sample-driven method on this instance
(every candidate from the d-spheres of the l-mers of s_1, tested against
s_2, s_3, ... until the first string without a hit; counted exactly by the
filter path) divided by the measured solve time of the fastest exact path,
with the input already in device memory.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_ALU_OPS = 256 * 64 * 2.4e9     # int32 VALU lane ops/s (256 CU x 64 x 2.4 GHz)
PEAK_HBM = 8.0e12                   # bytes/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_threads() -> int:
    n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, min(n, 16))


def cpu_baseline(inst, target_s: float = 12.0) -> dict:
    """The oracle as it stands, on a bounded sample of reference l-mers."""
    import oracle
    threads = host_threads()
    n, m, l, d = inst.n, inst.m, inst.l, inst.d
    L = m - l + 1
    # calibrate with one reference per thread, then size the sample
    k0 = min(L, threads)
    t0 = time.perf_counter()
    _, h0 = oracle.o1(inst.seqs, n, m, l, d, 0, k0, threads)
    t1 = time.perf_counter() - t0
    k = max(k0, min(L, int(k0 * target_s / max(t1, 1e-3))))
    k = max(threads, (k // threads) * threads)
    k = min(k, L)
    t0 = time.perf_counter()
    _, h = oracle.o1(inst.seqs, n, m, l, d, 0, k, threads)
    t = time.perf_counter() - t0
    return {"value": h / t, "unit": "Hamming tests/s", "cores": threads,
            "kind": "oracle",
            "sample": "sample-driven oracle over the first %d of %d reference "
                      "l-mers of s_1 (same instance), %.1f s, %d tests"
                      % (k, L, t, h)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not "
              "supported (multi-GPU sharding is described in DESIGN.md only)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2403_00306_amd as pms
    import pmsgen

    inst = pmsgen.plain("pms_17_6", args.seed)
    n, m, l, d = inst.n, inst.m, inst.l, inst.d
    dev = torch.device("cuda:0")
    d_seqs = torch.frombuffer(bytearray(inst.seqs), dtype=torch.uint8).to(dev)
    cap = 1 << 20
    d_out = torch.empty(cap, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()

    ctx = pms.Context(device=0)
    log("warmup", args.warmup)
    for _ in range(args.warmup):
        ctx.solve_device(d_seqs.data_ptr(), n, m, l, d, d_out.data_ptr(), cap)
    torch.cuda.synchronize()
    log("timed", args.steps)
    kms, stats = [], None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cnt = ctx.solve_device(d_seqs.data_ptr(), n, m, l, d,
                               d_out.data_ptr(), cap)
        stats = ctx.stats()
        kms.append(stats["ms_main"])
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ms_step = 1000.0 * t / args.steps
    motifs = d_out[:cnt].cpu().numpy().view(np.uint64)
    log("solve %.3f ms/step, kernel %.3f ms, %d motifs, path %s"
        % (ms_step, float(np.mean(kms)), cnt, stats["path_name"]))

    # canonical Hamming-test count from the filter path (exact count)
    fctx = pms.Context(device=0, path=pms.PATH_FILTER)
    fcnt = fctx.solve_device(d_seqs.data_ptr(), n, m, l, d, d_out.data_ptr(),
                             cap)
    fst = fctx.stats()
    fcodes = d_out[:fcnt].cpu().numpy().view(np.uint64)
    assert np.array_equal(fcodes, motifs), "filter and tiled paths disagree"
    hcanon = fst["hcanon"]
    log("filter path: %.1f ms kernel, H_canon %.4g" % (fst["ms_main"], hcanon))

    value = hcanon / (ms_step / 1000.0)
    k_ms = float(np.mean(kms))
    # dominant kernel of the timed path: algorithmic integer work
    L = m - l + 1
    alg_ops = (stats["marks"] * 2 + stats["tile_passes"] * L * 5 +
               stats["filter_tests"] * 4)
    achieved = alg_ops / (k_ms / 1000.0)
    roof = {"bound": "alu", "achieved": achieved / 1e12,
            "peak": PEAK_ALU_OPS / 1e12, "unit": "Tops/s",
            "frac": achieved / PEAK_ALU_OPS, "traffic": None,
            "kernel": "k_tiled", "kernel_ms": k_ms,
            "ops_per_launch": alg_ops}
    f_ops = hcanon * 3.5
    roof_filter = {"bound": "alu", "kernel": "k_filter",
                   "kernel_ms": fst["ms_main"],
                   "tests_per_s": hcanon / (fst["ms_main"] / 1000.0),
                   "achieved": f_ops / (fst["ms_main"] / 1000.0) / 1e12,
                   "peak": PEAK_ALU_OPS / 1e12, "unit": "Tops/s",
                   "frac": f_ops / (fst["ms_main"] / 1000.0) / PEAK_ALU_OPS}
    extra = {}
    if not args.no_extra:
        bctx = pms.Context(device=0, path=pms.PATH_BITSET)
        bcnt = bctx.solve_device(d_seqs.data_ptr(), n, m, l, d,
                                 d_out.data_ptr(), cap)
        bst = bctx.stats()
        bcodes = d_out[:bcnt].cpu().numpy().view(np.uint64)
        assert np.array_equal(bcodes, motifs), "bitset path disagrees"
        extra["memory_heavy_bitset_path"] = {
            "solve_ms": bst["ms_total"], "kernel_ms": bst["ms_main"],
            "bitset_bytes": 4 ** l // 8, "hbm_bytes": bst["bytes_main"],
            "hbm_GBps": bst["bytes_main"] / (bst["ms_main"] / 1000.0) / 1e9,
            "frac_hbm": bst["bytes_main"] / (bst["ms_main"] / 1000.0)
            / PEAK_HBM}
        bctx.close()
    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline(inst)
        log("cpu %.4g tests/s on %d threads" % (cpu["value"], cpu["cores"]))

    rec = {"metric": "Hamming tests/s", "value": value,
           "unit": "Hamming tests/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u32", "data": "synthetic",
           "config": {"workload": "planted (17,6) motif search, n=20 "
                      "strings, m=600, seed %d" % args.seed,
                      "n": n, "m": m, "l": l, "d": d,
                      "path": stats["path_name"],
                      "tile_suffix": stats["tile_suffix"]},
           "solve_ms_17_6": ms_step, "motifs": int(cnt),
           "hcanon": int(hcanon),
           "roofline": roof, "roofline_filter": roof_filter,
           "cpu_baseline": cpu}
    rec.update(extra)
    print(json.dumps(rec), flush=True)
    fctx.close()
    ctx.close()


if __name__ == "__main__":
    main()
