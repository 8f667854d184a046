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

# Algorithmic integer operations per unit of work (gfx950 forms):
#  Hamming test on bit planes: v_xor + v_bitop3 (xor, or) + v_bcnt + half a
#    v_min3 = 3.5
#  tile prefix test: xor + bitop3 + and + bcnt, compare folded = 4
#  word-level sphere mark: word index xor + the OR itself = 2
OPS_TEST = 3.5
# the calibration kernel's loop body as compiled for gfx950: per 128 tests
# 128 v_xor, 128 v_bitop3, 128 v_bcnt, 64 v_min and 32 v_min3
VALU_PER_TEST_CAL = 480.0 / 128.0
OPS_PREFIX = 4.0
OPS_MARK = 2.0
# any-alphabet filter, per Hamming test on 5 bit planes: v_xor, four
#   v_bitop3 (s0 | (s1 ^ s2)), v_bcnt and half a v_min3 = 6.5
OPS_TEST_ALPHA = 6.5
# long motifs (l up to 64), per Hamming test on two 64-bit planes: per
#   32-bit half a v_xor, a v_bitop3 and a v_bcnt, then half a v_min = 6.5
OPS_TEST_WIDE = 6.5
# quorum path, per 64-code word per pass: the bit-sliced increment (XOR and
# AND per counter plane, 5 planes); counters start at 31 - (n - q), so the
# carry out of the top plane is the test and needs no compare
OPS_COUNT = 10.0
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "pms_17_6_traffic.json")


def tile_kernel(st) -> str:
    """Name of the tile kernel a plain tiled solve ran (its stats)."""
    return "k_tiled_512" if st.get("tile_threads") == 512 else "k_tiled"


def measured_traffic(kernel: str, pick: str = "bytes"):
    """HBM bytes per dispatch from the committed counter profile, if it was
    taken on the current source of that kernel (else None). pick: "bytes"
    (mean over dispatches), "min_bytes" or "max_bytes" (for a kernel that
    the profiled run launches on two workload sizes)."""
    try:
        from paper_2403_00306_amd import profile_tools
        rec = json.load(open(TRAFFIC_JSON))["kernels"][kernel]
        if rec["source_sha"] == profile_tools.source_hash(kernel):
            return rec[pick]
    except (OSError, KeyError, ValueError):
        pass
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def usable_cpus() -> int:
    """CPUs this process may run on (its affinity mask)."""
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def host_threads() -> int:
    """Threads the oracle runs on: every CPU this process may use, at most
    OMP_NUM_THREADS when that is set."""
    n = usable_cpus()
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def cpu_model() -> str:
    """The host CPU's model name as lscpu reports it (else /proc/cpuinfo)."""
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True,
                             timeout=10).stdout
        for line in out.splitlines():
            if line.strip().startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def single_thread_oracle(pmsgen) -> dict:
    """The oracle on one thread: all of (9,2) and the first 30 reference
    l-mers of (13,4) (n = 20, m = 600, seed 1)."""
    import oracle
    out = {}
    for name, l, d, refs in (("pms_9_2", 9, 2, None), ("pms_13_4", 13, 4, 30)):
        inst = pmsgen.plain(name, 1)
        L = inst.m - l + 1
        k = L if refs is None else min(refs, L)
        t0 = time.perf_counter()
        _, h = oracle.o1(inst.seqs, inst.n, inst.m, l, d, 0, k, 1)
        t = time.perf_counter() - t0
        out[name] = {"tests_per_s": h / t, "seconds": t, "tests": int(h),
                     "references": "%d of %d" % (k, L)}
    return out


def seeds_bench(pms, pmsgen, np) -> dict:
    """(17,6), n = 20, m = 600, seeds 1..5: wall time of pms_solve from host
    bytes to the host sorted set on a warm context, median of 3 (tiled path,
    with its kernel time), and one filter-path solve per seed."""
    res = {}
    tctx = pms.Context(device=0, path=pms.PATH_TILED)
    fctx = pms.Context(device=0, path=pms.PATH_FILTER)
    for seed in range(1, 6):
        inst = pmsgen.planted(seed, 20, 600, 17, 6)
        tctx.solve(inst.seqs, 20, 600, 17, 6)            # warm
        walls, kms = [], []
        for _ in range(3):
            t0 = time.perf_counter()
            got = tctx.solve(inst.seqs, 20, 600, 17, 6)
            walls.append((time.perf_counter() - t0) * 1000.0)
            kms.append(tctx.stats()["ms_main"])
        t0 = time.perf_counter()
        fgot = fctx.solve(inst.seqs, 20, 600, 17, 6)
        fwall = (time.perf_counter() - t0) * 1000.0
        assert np.array_equal(got, fgot), "paths disagree at seed %d" % seed
        res["seed_%d" % seed] = {
            "tiled_solve_ms": float(np.median(walls)),
            "tiled_kernel_ms": float(np.median(kms)),
            "filter_solve_ms": fwall,
            "filter_kernel_ms": fctx.stats()["ms_main"],
            "motifs": int(len(got))}
    tctx.close()
    fctx.close()
    log("seeds: " + json.dumps(res))
    return res


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
            "kind": "oracle", "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(), "usable_cpus": usable_cpus(),
            "threads_rule": "every CPU in the process's affinity mask, at "
                            "most OMP_NUM_THREADS when set",
            "sample": "sample-driven oracle over the first %d of %d reference "
                      "l-mers of s_1 (same instance), %.1f s, %d tests"
                      % (k, L, t, h)}


GOLDEN = os.path.join(ROOT, "tests", "golden")


def oracle_checked(np, name: str, insts, results) -> dict:
    """Compare GPU motif sets with the exact sets the oracle stored in
    tests/golden/<name> (index n m l d input_sha count hcanon codes_sha
    codes): the instance's shape and input hash must match, then the count
    and the hash of the ascending codes (and the codes themselves where
    stored). Instances without a stored set are not counted."""
    import hashlib
    path = os.path.join(GOLDEN, name)
    stored = {}
    try:
        for line in open(path):
            if not line.strip() or line.startswith("#") or "=" in line:
                continue
            t = line.split()
            stored[int(t[0])] = t
    except OSError:
        return {"file": "tests/golden/" + name, "stored": 0, "checked": 0,
                "matched": 0}
    checked = matched = 0
    for i, (x, got) in enumerate(zip(insts, results)):
        t = stored.get(i)
        if t is None:
            continue
        checked += 1
        got = np.asarray(got, dtype=np.uint64)
        ok = ((int(t[1]), int(t[2]), int(t[3]), int(t[4])) ==
              (x.n, x.m, x.l, x.d) and
              hashlib.sha256(x.seqs).hexdigest() == t[5] and
              len(got) == int(t[6]) and
              hashlib.sha256(got.astype("<u8").tobytes()).hexdigest() == t[8])
        if ok and t[9] not in ("-", "none"):
            ok = got.tolist() == [int(v) for v in t[9].split(",")]
        matched += bool(ok)
    return {"file": "tests/golden/" + name, "stored": len(stored),
            "instances": len(insts), "checked": checked, "matched": matched,
            "fraction_checked": checked / max(1, len(insts))}


def oracle_refs_checked(name: str, insts, results) -> dict:
    """Requests with stored reference subsets (tests/golden/<name>: index l
    d j input_sha hcanon count codes, the motifs the oracle derives from one
    reference l-mer of s_1): each subset must lie in the served set."""
    import hashlib
    per = {}
    try:
        for line in open(os.path.join(GOLDEN, name)):
            if not line.strip() or line.startswith("#"):
                continue
            t = line.split()
            codes = [] if t[7] == "none" else [int(v) for v in t[7].split(",")]
            per.setdefault(int(t[0]), []).append((t[4], codes))
    except OSError:
        return {"file": "tests/golden/" + name, "requests": 0, "matched": 0}
    matched = 0
    for i, subsets in per.items():
        x, got = insts[i], set(int(v) for v in results[i])
        matched += all(hashlib.sha256(x.seqs).hexdigest() == sha and
                       set(codes) <= got for sha, codes in subsets)
    return {"file": "tests/golden/" + name, "requests": len(per),
            "references": sum(len(v) for v in per.values()),
            "matched": matched}


def batch_bench(pms, pmsgen, np, tune: bool) -> dict:
    """256 independent instances: one pms_solve_batch call (one persistent
    launch, replayed as a HIP graph) vs the same instances solved one by
    one with pms_solve, on the same context."""
    insts = pmsgen.batched(seed=7, count=256)
    ctx = pms.Context(device=0)
    t_tune = 0.0
    if tune:
        t0 = time.perf_counter()
        seen = set()
        for x in insts:
            key = (x.l, x.d, x.n.bit_length(), x.m.bit_length())
            if key not in seen:
                seen.add(key)
                ctx.autotune(x.n, x.m, x.l, x.d)
        t_tune = time.perf_counter() - t0
    ctx.solve_batch(insts)                       # warm-up + graph capture
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        got = ctx.solve_batch(insts)
    t_batch = (time.perf_counter() - t0) / reps
    bst = ctx.stats()
    t0 = time.perf_counter()
    alone = [ctx.solve(x.seqs, x.n, x.m, x.l, x.d) for x in insts]
    t_plain = time.perf_counter() - t0
    same = all(np.array_equal(a, b) for a, b in zip(got, alone))
    ctx.close()
    return {"instances": len(insts), "batched_instances_per_s":
            len(insts) / t_batch, "plain_instances_per_s":
            len(insts) / t_plain, "batched_ms": 1000 * t_batch,
            "plain_ms": 1000 * t_plain, "batch_kernel_ms": bst["ms_main"],
            "motifs_total": int(sum(len(a) for a in alone)),
            "batched_equals_plain": bool(same), "autotune_s": t_tune,
            "oracle_checked": oracle_checked(np, "batched_seed7.txt", insts,
                                             got)}


def quorum_bench(pms, pmsgen, np, torch, dev, reps: int = 3) -> dict:
    """(l,d,q)-motifs at the thesis's q = 10 shape (n = 20, m = 600):
    device-resident solve time and the quorum kernel's roofline."""
    res = {}
    for name, q in (("pms_13_4", 10), ("pms_17_6", 10)):
        inst = pmsgen.plain(name, 1)
        n, m, l, d = inst.n, inst.m, inst.l, inst.d
        d_seqs = torch.frombuffer(bytearray(inst.seqs),
                                  dtype=torch.uint8).to(dev)
        ctx = pms.Context(device=0)
        cap = 1 << 16
        d_out = torch.empty(cap, dtype=torch.int64, device=dev)
        try:
            ctx.solve_quorum_device(d_seqs.data_ptr(), n, m, l, d, q,
                                    d_out.data_ptr(), cap)
        except pms.PmsError as e:
            cap = e.needed
            del d_out
            d_out = torch.empty(cap, dtype=torch.int64, device=dev)
        ctx.solve_quorum_device(d_seqs.data_ptr(), n, m, l, d, q,
                                d_out.data_ptr(), cap)
        torch.cuda.synchronize()
        walls, kms = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            cnt = ctx.solve_quorum_device(d_seqs.data_ptr(), n, m, l, d, q,
                                          d_out.data_ptr(), cap)
            walls.append((time.perf_counter() - t0) * 1000.0)
            st = ctx.stats()
            kms.append(st["ms_main"])
        k_ms = float(np.mean(kms))
        L = m - l + 1
        words = 4 ** (st["tile_suffix"] - 3)
        ops = (st["marks"] * OPS_MARK + st["tile_passes"] * L * OPS_PREFIX +
               st["tile_passes"] * words * OPS_COUNT)
        achieved = ops / (k_ms / 1000.0)
        res["%s_q%d" % (name, q)] = {
            "workload": "(%d,%d,%d)-motifs, n=%d, m=%d, seed 1"
                        % (l, d, q, n, m),
            "motifs": int(cnt), "solve_ms": min(walls), "kernel_ms": k_ms,
            "output_ms": st["ms_output"], "tiles": st["tiles"],
            "passes": st["tile_passes"], "tile_suffix": st["tile_suffix"],
            "roofline": {"bound": "alu", "kernel": "k_tiled_quorum",
                         "achieved": achieved / 1e12,
                         "peak": PEAK_ALU_OPS / 1e12, "unit": "TOP/s",
                         "frac": achieved / PEAK_ALU_OPS,
                         # the profiled run launches it at (13,4), then
                         # at (17,6): smallest and largest dispatches
                         "traffic": measured_traffic(
                             "k_tiled_quorum",
                             "max_bytes" if l >= 17 else "min_bytes"),
                         "ops_per_launch": ops}}
        log("quorum %s q=%d: %d motifs, %.2f ms solve, %.2f ms kernel"
            % (name, q, cnt, min(walls), k_ms))
        ctx.close()
        del d_out, d_seqs
        torch.cuda.empty_cache()
    return res


def hard_bench(pms, pmsgen, np) -> dict:
    """The thesis's harder planted instances (Table 3.3 shapes, n = 20,
    m = 600, seed 1) on the tiled path: solve time and k_tiled's roofline."""
    res = {}
    for l, d in ((19, 7), (21, 8), (23, 9)):
        inst = pmsgen.planted(1, 20, 600, l, d)
        with pms.Context(device=0, path=pms.PATH_TILED) as c:
            t0 = time.perf_counter()
            got = c.solve(inst.seqs, 20, 600, l, d)
            wall = (time.perf_counter() - t0) * 1000.0
            st = c.stats()
        L = 600 - l + 1
        ops = (st["marks"] * OPS_MARK + st["tile_passes"] * L * OPS_PREFIX +
               st["filter_tests"] * OPS_TEST)
        plant = 0
        for ch in inst.motif:
            plant = 4 * plant + b"ACGT".index(ch)
        res["pms_%d_%d" % (l, d)] = {
            "workload": "planted (%d,%d), n=20, m=600, seed 1" % (l, d),
            "solve_ms": wall, "kernel_ms": st["ms_main"],
            "motifs": int(len(got)),
            "planted_found": bool(plant in set(int(v) for v in got)),
            "tiles": st["tiles"], "passes": st["tile_passes"],
            "roofline": {"bound": "alu", "kernel": tile_kernel(st),
                         "achieved": ops / (st["ms_main"] / 1000.0) / 1e12,
                         "peak": PEAK_ALU_OPS / 1e12, "unit": "TOP/s",
                         "frac": ops / (st["ms_main"] / 1000.0)
                         / PEAK_ALU_OPS}}
        log("hard (%d,%d): %.1f ms, %d motifs" % (l, d, wall, len(got)))
    return res


def protein_bench(pms, pmsgen, np) -> dict:
    """Planted instances over the 20 amino-acid letters (n = 20, m = 600,
    seed 1): the any-alphabet sample-driven filter; canonical Hamming tests
    per second and its roofline (5 XOR, 4 OR, popcount and compare per test
    on 5 bit planes)."""
    res = {}
    with pms.Context(device=0) as c:
        for l, d in ((9, 3), (10, 4)):
            inst = pmsgen.planted_alpha(1, 20, 600, l, d)
            c.solve_alphabet(pmsgen.PROTEIN, inst.seqs, 20, 600, l, d)
            t0 = time.perf_counter()
            got = c.solve_alphabet(pmsgen.PROTEIN, inst.seqs, 20, 600, l, d)
            wall = (time.perf_counter() - t0) * 1000.0
            st = c.stats()
            plant = 0
            for ch in inst.motif:
                plant = plant * 20 + pmsgen.PROTEIN.index(ch)
            ops = st["hcanon"] * OPS_TEST_ALPHA
            res["protein_%d_%d" % (l, d)] = {
                "workload": "planted (%d,%d) over 20 letters, n=20, m=600, "
                            "seed 1" % (l, d),
                "solve_ms": wall, "kernel_ms": st["ms_main"],
                "motifs": int(len(got)),
                "planted_found": bool(plant in set(int(v) for v in got)),
                "hcanon": st["hcanon"],
                "tests_per_s": st["hcanon"] / (st["ms_main"] / 1000.0),
                "roofline": {"bound": "alu", "kernel": "k_alpha_filter",
                             # profiled at (9,3), then (10,4)
                             "traffic": measured_traffic(
                                 "k_alpha_filter",
                                 "max_bytes" if l >= 10 else "min_bytes"),
                             "achieved": ops / (st["ms_main"] / 1000.0) / 1e12,
                             "peak": PEAK_ALU_OPS / 1e12, "unit": "TOP/s",
                             "frac": ops / (st["ms_main"] / 1000.0)
                             / PEAK_ALU_OPS}}
            log("protein (%d,%d): %.1f ms, %d motifs" % (l, d, wall, len(got)))
    return res


def wide_bench(pms, pmsgen, np) -> dict:
    """Long motifs: planted (40,4), n = 20, m = 600, seed 1, through the
    128-bit-code path (one 64-bit word per bit plane); canonical Hamming
    tests per second and its roofline."""
    inst = pmsgen.planted(1, 20, 600, 40, 4)
    plant = 0
    for ch in inst.motif:
        plant = 4 * plant + b"ACGT".index(ch)
    with pms.Context(device=0) as c:
        c.solve_wide(inst.seqs, 20, 600, 40, 4)
        t0 = time.perf_counter()
        got = c.solve_wide(inst.seqs, 20, 600, 40, 4)
        wall = (time.perf_counter() - t0) * 1000.0
        st = c.stats()
    codes = set((int(h) << 64) | int(lo) for h, lo in got)
    ops = st["hcanon"] * OPS_TEST_WIDE
    log("wide (40,4): %.1f ms, %d motifs" % (wall, len(got)))
    return {"workload": "planted (40,4), n=20, m=600, seed 1",
            "solve_ms": wall, "kernel_ms": st["ms_main"],
            "motifs": int(len(got)), "planted_found": plant in codes,
            "hcanon": st["hcanon"],
            "tests_per_s": st["hcanon"] / (st["ms_main"] / 1000.0),
            "roofline": {"bound": "alu", "kernel": "k_wide_filter",
                         "traffic": measured_traffic("k_wide_filter"),
                         "achieved": ops / (st["ms_main"] / 1000.0) / 1e12,
                         "peak": PEAK_ALU_OPS / 1e12, "unit": "TOP/s",
                         "frac": ops / (st["ms_main"] / 1000.0)
                         / PEAK_ALU_OPS}}


def pair_bench(pms, inst, np) -> dict:
    """The pair-based sample-driven path (Observation 3.3) on the timed
    (17,6) instance: compatible pairs, candidates, tests and its roofline."""
    with pms.Context(device=0, path=pms.PATH_PAIR) as c:
        c.solve(inst.seqs, inst.n, inst.m, inst.l, inst.d)
        t0 = time.perf_counter()
        got = c.solve(inst.seqs, inst.n, inst.m, inst.l, inst.d)
        wall = (time.perf_counter() - t0) * 1000.0
        st = c.stats()
    ops = st["filter_tests"] * OPS_TEST
    log("pair path (17,6): %.1f ms, %d pairs, %.4g candidates"
        % (wall, st["pairs"], st["candidates"]))
    return {"solve_ms": wall, "kernel_ms": st["ms_main"],
            "motifs": int(len(got)), "pairs": st["pairs"],
            "candidates": st["candidates"], "tests": st["filter_tests"],
            "roofline": {"bound": "alu", "kernel": "k_pair_filter",
                         "traffic": measured_traffic("k_pair_filter"),
                         "achieved": ops / (st["ms_main"] / 1000.0) / 1e12,
                         "peak": PEAK_ALU_OPS / 1e12, "unit": "TOP/s",
                         "frac": ops / (st["ms_main"] / 1000.0) / PEAK_ALU_OPS}}


def serve_bench(pms, pmsgen, np, count: int, launch_ms: float = 0.0) -> dict:
    """Poisson request stream through the continuous-batching engine:
    first a saturation pass (all requests at t=0) gives the capacity C;
    then an open-loop pass at rate 0.8*C reports p50/p99 latency."""
    reqs = pmsgen.served(seed=11, count=count)

    def run(rate):
        ctx = pms.Context(device=0, serve_slots=64, serve_launch_ms=launch_ms)
        t_start = ctx.clock_ms()
        tickets = []
        for r in reqs:
            if rate:
                due = t_start + 1000.0 * r.arrival_unit / rate
                while ctx.clock_ms() < due:
                    time.sleep(max(0.0, (due - ctx.clock_ms()) / 1000.0 - 2e-4))
            x = r.inst
            tickets.append((ctx.submit(x.seqs, x.n, x.m, x.l, x.d),
                            t_start + (1000.0 * r.arrival_unit / rate
                                       if rate else 0.0)))
        results, lat = [], []
        t_last = t_start
        for tk, t_arr in tickets:
            res = ctx.wait(tk, 600000)
            ts, ta, td = ctx.ticket_times(tk)
            lat.append(td - t_arr)      # completion - (scheduled) arrival
            t_last = max(t_last, td)
            results.append(res)
            ctx.release(tk)
        st = ctx.serve_stats()
        ctx.close()
        return results, np.array(lat), (t_last - t_start) / 1000.0, st

    res_sat, lat_sat, span_sat, st_sat = run(0.0)
    cap = len(reqs) / span_sat
    rate = 0.8 * cap
    res, lat, span, st = run(rate)
    same = all(np.array_equal(a, b) for a, b in zip(res, res_sat))
    # a sample solved alone must equal its served result
    ctx = pms.Context(device=0)
    idx = list(range(0, len(reqs), max(1, len(reqs) // 50)))
    alone_ok = all(np.array_equal(ctx.solve(reqs[i].inst.seqs, reqs[i].inst.n,
                                            reqs[i].inst.m, reqs[i].inst.l,
                                            reqs[i].inst.d), res[i])
                   for i in idx)
    ctx.close()
    return {"requests": len(reqs), "capacity_instances_per_s": cap,
            "rate_per_s": rate, "instances_per_s": len(reqs) / span,
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "saturation_p50_ms": float(np.percentile(lat_sat, 50)),
            "max_inflight": int(st["max_inflight"]),
            "launches": int(st["launches"]),
            "launch_ms_target": launch_ms or None,
            "mix_equals_saturated_and_alone": bool(same and alone_ok),
            "oracle_checked": oracle_checked(
                np, "served_seed11.txt", [r.inst for r in reqs], res),
            "oracle_refs_checked": oracle_refs_checked(
                "served_seed11_refs.txt", [r.inst for r in reqs], res)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-hard", action="store_true",
                    help="skip the (19,7)/(21,8)/(23,9) leg (~17 s)")
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--serve-launch-ms", type=float, default=0.0,
                    help="device time each serving launch aims at "
                         "(0: the library default)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="MiB: one device copy of this size at the end, to "
                         "calibrate rocprofv3 FETCH_SIZE/WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU per process; --gpus %d "
              "is not supported (sharding across GPUs is a design, not "
              "code)" % args.gpus, file=sys.stderr)
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
    # dominant kernel of the timed path (k_tiled or, for tiles of 4^8-4^9 codes,
    # its 512-thread form k_tiled_512): algorithmic integer work
    # of one launch from its work counters, over its average HIP-event time
    L = m - l + 1
    alg_ops = (stats["marks"] * OPS_MARK +
               stats["tile_passes"] * L * OPS_PREFIX +
               stats["filter_tests"] * OPS_TEST)
    achieved = alg_ops / (k_ms / 1000.0)
    roof = {"bound": "alu", "achieved": achieved / 1e12,
            "peak": PEAK_ALU_OPS / 1e12, "unit": "TOP/s",
            "frac": achieved / PEAK_ALU_OPS,
            "traffic": measured_traffic(tile_kernel(stats)),
            "kernel": tile_kernel(stats), "kernel_ms": k_ms,
            "ops_per_launch": alg_ops, "marks": stats["marks"],
            "prefix_tests": stats["tile_passes"] * L,
            "filter_tests": stats["filter_tests"]}
    # the same kernel against the LDS: its marks are single-bit or mask ORs
    # into the tile in LDS and every pass reads and clears the tile's words
    # once; the peak is the device's measured rate of that OR (calibration
    # kernel at the same occupancy)
    cal_lds = pms.Context(device=0)
    lds_peak = cal_lds.lds_rate()
    cal_lds.close()
    words_per_tile = 4 ** (stats["tile_suffix"] - 3)
    lds_ops = stats["marks"] + stats["tile_passes"] * words_per_tile
    roof_lds = {"bound": "lds", "kernel": tile_kernel(stats),
                "achieved": lds_ops / (k_ms / 1000.0) / 1e12,
                "peak": lds_peak / 1e12, "unit": "T lane-ops/s",
                "frac": lds_ops / (k_ms / 1000.0) / lds_peak,
                "lane_ops_per_launch": lds_ops,
                "peak_source": "pms_lds_rate: single-bit LDS atomic ORs, "
                               "512-thread workgroups, 32 KiB LDS each"}
    log("lds: %.3g lane-ops/s of %.3g measured peak (%.3f)"
        % (lds_ops / (k_ms / 1000.0), lds_peak, roof_lds["frac"]))
    f_ops = hcanon * OPS_TEST
    roof_filter = {"bound": "alu", "kernel": "k_filter",
                   "kernel_ms": fst["ms_main"],
                   "tests_per_s": hcanon / (fst["ms_main"] / 1000.0),
                   "achieved": f_ops / (fst["ms_main"] / 1000.0) / 1e12,
                   "peak": PEAK_ALU_OPS / 1e12, "unit": "TOP/s",
                   "frac": f_ops / (fst["ms_main"] / 1000.0) / PEAK_ALU_OPS,
                   "traffic": measured_traffic("k_filter"),
                   # the tests the kernel executed (whole waves, including
                   # empty candidate slots) and the same fraction on them
                   "exec_tests": fst["filter_tests"],
                   "frac_exec": fst["filter_tests"] * OPS_TEST
                   / (fst["ms_main"] / 1000.0) / PEAK_ALU_OPS}
    extra = {}
    if not args.no_extra:
        bctx = pms.Context(device=0, path=pms.PATH_BITSET)
        # the first call allocates the 4^l-bit set; time the second
        for _ in range(2):
            bcnt = bctx.solve_device(d_seqs.data_ptr(), n, m, l, d,
                                     d_out.data_ptr(), cap)
        bst = bctx.stats()
        bcodes = d_out[:bcnt].cpu().numpy().view(np.uint64)
        assert np.array_equal(bcodes, motifs), "bitset path disagrees"
        bw = bst["bytes_main"] / (bst["ms_main"] / 1000.0)
        extra["memory_heavy_bitset_path"] = {
            "solve_ms": bst["ms_total"], "kernel_ms": bst["ms_main"],
            "launches": bst["main_launches"], "bitset_bytes": 4 ** l // 8,
            "tile_passes": bst["tile_passes"], "marks": bst["marks"],
            "marks_per_s": bst["marks"] / (bst["ms_main"] / 1000.0),
            "roofline": {"bound": "hbm", "achieved": bw / 1e9,
                         "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                         "frac": bw / PEAK_HBM,
                         "traffic": measured_traffic("k_bitset_pass"),
                         "algorithmic_bytes": bst["bytes_main"]}}
        bctx.close()
        # the filter's Hamming-test mix at full occupancy from registers:
        # a check of the derived integer peak the roofline figures use
        cal = pms.Context(device=0)
        rate = cal.test_rate()
        cal.close()
        extra["alu_calibration"] = {
            "tests_per_s": rate,
            "valu_per_test_in_loop": VALU_PER_TEST_CAL,
            "valu_lane_ops_per_s": rate * VALU_PER_TEST_CAL,
            "derived_peak_ops_per_s": PEAK_ALU_OPS,
            "frac_of_derived_peak": rate * VALU_PER_TEST_CAL / PEAK_ALU_OPS}
        log("alu calibration: %.4g tests/s, %.3g of the derived peak"
            % (rate, extra["alu_calibration"]["frac_of_derived_peak"]))
        extra["seeds_17_6"] = seeds_bench(pms, pmsgen, np)
        extra["quorum"] = quorum_bench(pms, pmsgen, np, torch, dev)
        extra["pair_path"] = pair_bench(pms, inst, np)
        extra["protein"] = protein_bench(pms, pmsgen, np)
        extra["wide"] = wide_bench(pms, pmsgen, np)
        if not args.no_hard:
            extra["hard"] = hard_bench(pms, pmsgen, np)
    if not args.no_batch:
        log("batched")
        extra["batched"] = batch_bench(pms, pmsgen, np, not args.no_tune)
        log(json.dumps(extra["batched"]))
    if not args.no_serve:
        log("served")
        extra["served"] = serve_bench(pms, pmsgen, np, args.serve_count,
                                      args.serve_launch_ms)
        log(json.dumps(extra["served"]))
    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline(inst)
        if not args.no_extra:
            cpu["single_thread"] = single_thread_oracle(pmsgen)
        log("cpu %.4g tests/s on %d threads" % (cpu["value"], cpu["cores"]))

    rec = {"metric": "Hamming tests/s", "value": value,
           "unit": "Hamming tests/s",
           "value_kind": "canonical-equivalent: the sample-driven method's "
                         "exact Hamming-test count H_canon of this instance "
                         "(counted by the filter path) divided by the "
                         "fastest exact path's solve time (tiled: marks plus "
                         "%d executed tests); the filter path's own rate is "
                         "roofline_filter.tests_per_s" % stats["filter_tests"],
           "n_gpus": 1, "steps": args.steps,
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
           "roofline": roof, "roofline_lds": roof_lds,
           "roofline_filter": roof_filter,
           "cpu_baseline": cpu}
    rec.update(extra)
    if args.copy_probe:
        a = torch.empty(args.copy_probe << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    print(json.dumps(rec), flush=True)
    fctx.close()
    ctx.close()


if __name__ == "__main__":
    main()
