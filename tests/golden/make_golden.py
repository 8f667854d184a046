"""Write the stored full-size results used by tests/test_oracle.py.

Calls only the CPU oracle (both O1 and the brute force O0, which must agree)
on inputs from the seeded generator; nothing here touches the GPU library.
Run from the repository root:  python tests/golden/make_golden.py
(add "quorum" or "protein" to write only those files; "large", "batched",
"served", "served_refs", "hard" or "wide" write the long-running sets
below, which take hours of CPU time and resume where an interrupted run
stopped)
"""
import hashlib
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import pmsgen  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = [("pms_9_2", 1), ("pms_9_2", 2), ("pms_9_2", 3), ("pms_13_4", 1)]
# quorum (l,d,q)-motif sets: Q1 and the brute force Q0 must agree; the set
# is stored as its size and the hash of its codes (little-endian uint64)
QCASES = [("pms_9_2", 1, 10), ("pms_9_2", 1, 15), ("pms_9_2", 2, 5)]


def main():
    for name, seed in CASES:
        inst = pmsgen.plain(name, seed)
        t0 = time.time()
        o1, h = oracle.o1(inst.seqs, inst.n, inst.m, inst.l, inst.d)
        t1 = time.time()
        o0 = oracle.o0(inst.seqs, inst.n, inst.m, inst.l, inst.d)
        t2 = time.time()
        assert list(o1) == list(o0), (name, seed)
        path = os.path.join(HERE, "%s_seed%d.txt" % (name, seed))
        with open(path, "w") as f:
            f.write("# Exact (l,d)-motif set of one synthetic planted instance,\n")
            f.write("# written by tests/golden/make_golden.py from the CPU oracle\n")
            f.write("# (sample-driven O1 and brute-force O0 agree).\n")
            f.write("config = %s\nseed = %d\n" % (name, seed))
            f.write("n = %d\nm = %d\nl = %d\nd = %d\n"
                    % (inst.n, inst.m, inst.l, inst.d))
            f.write("input_sha256 = %s\n" % hashlib.sha256(inst.seqs).hexdigest())
            f.write("planted = %s\n" % inst.motif.decode())
            f.write("hcanon = %d\n" % h)
            f.write("count = %d\n" % len(o1))
            f.write("motifs = %s\n" % ",".join(str(int(v)) for v in o1))
            f.write("motif_strings = %s\n" % ",".join(
                oracle.decode_code(v, inst.l).decode() for v in o1))
        print(name, seed, len(o1), "O1 %.1fs O0 %.1fs" % (t1 - t0, t2 - t1))


def main_quorum():
    for name, seed, q in QCASES:
        inst = pmsgen.plain(name, seed)
        q1 = oracle.q1(inst.seqs, inst.n, inst.m, inst.l, inst.d, q)
        q0 = oracle.q0(inst.seqs, inst.n, inst.m, inst.l, inst.d, q)
        assert list(q1) == list(q0), (name, seed, q)
        path = os.path.join(HERE, "%s_seed%d_q%d.txt" % (name, seed, q))
        with open(path, "w") as f:
            f.write("# Exact (l,d,q)-motif set of one synthetic planted instance,\n")
            f.write("# written by tests/golden/make_golden.py from the CPU oracle\n")
            f.write("# (Q1, Observation 3.1, and brute-force Q0 agree).\n")
            f.write("config = %s\nseed = %d\nq = %d\n" % (name, seed, q))
            f.write("n = %d\nm = %d\nl = %d\nd = %d\n"
                    % (inst.n, inst.m, inst.l, inst.d))
            f.write("input_sha256 = %s\n" % hashlib.sha256(inst.seqs).hexdigest())
            f.write("count = %d\n" % len(q1))
            f.write("codes_sha256 = %s\n" % hashlib.sha256(
                q1.astype("<u8").tobytes()).hexdigest())
            f.write("first = %s\n" % ",".join(str(int(v)) for v in q1[:8]))
            f.write("last = %s\n" % ",".join(str(int(v)) for v in q1[-8:]))
        print(name, seed, q, len(q1))


# other alphabets: the protein alphabet at (8,3), n = 20, m = 600 (S1 only:
# the 20^8 space is beyond the brute force)
PCASES = [(1, 8, 3)]


def main_protein():
    for seed, l, d in PCASES:
        inst = pmsgen.planted_alpha(seed, 20, 600, l, d)
        t0 = time.time()
        got = oracle.s1(inst.seqs, pmsgen.PROTEIN, 20, 600, l, d)
        plant = 0
        for ch in inst.motif:
            plant = plant * 20 + pmsgen.PROTEIN.index(ch)
        path = os.path.join(HERE, "protein_%d_%d_seed%d.txt" % (l, d, seed))
        with open(path, "w") as f:
            f.write("# Exact (l,d)-motif set of one synthetic planted protein\n")
            f.write("# instance, written by tests/golden/make_golden.py from the\n")
            f.write("# CPU oracle S1 (codes in base 20 over the alphabet below).\n")
            f.write("alphabet = %s\nseed = %d\n" % (pmsgen.PROTEIN.decode(), seed))
            f.write("n = 20\nm = 600\nl = %d\nd = %d\n" % (l, d))
            f.write("input_sha256 = %s\n" % hashlib.sha256(inst.seqs).hexdigest())
            f.write("planted = %s\nplanted_code = %d\n" % (inst.motif.decode(), plant))
            f.write("count = %d\n" % len(got))
            f.write("motifs = %s\n" % ",".join(str(int(v)) for v in got))
        print("protein", seed, l, d, len(got), "%.1fs" % (time.time() - t0))


# ---------------------------------------------------------------------------
# Long runs: the (17,6) configuration, more seeds of the small ones, the
# 256-instance batch, a sample of the served stream and sampled reference
# l-mers of the harder instances. Every set comes from O1 alone (O0 is out of
# reach above l = 13); at (9,2) and (13,4) O0 must agree as above.
# ---------------------------------------------------------------------------

THREADS = int(os.environ.get("GOLDEN_THREADS", "0"))   # 0 = every core
# (17,6) seeds 1..5; more seeds of (9,2) and (13,4)
LARGE = [("pms_9_2", 4), ("pms_9_2", 5), ("pms_13_4", 2), ("pms_13_4", 3),
         ("pms_13_4", 4), ("pms_13_4", 5), ("pms_17_6", 1), ("pms_17_6", 2),
         ("pms_17_6", 3), ("pms_17_6", 4), ("pms_17_6", 5),
         ("pms_19_7", 1)]


def main_large():
    for name, seed in LARGE:
        path = os.path.join(HERE, "%s_seed%d.txt" % (name, seed))
        if os.path.exists(path):
            continue
        inst = pmsgen.plain(name, seed)
        t0 = time.time()
        o1, h = oracle.o1(inst.seqs, inst.n, inst.m, inst.l, inst.d,
                          threads=THREADS)
        t1 = time.time()
        both = inst.l <= 13
        if both:
            o0 = oracle.o0(inst.seqs, inst.n, inst.m, inst.l, inst.d,
                           threads=THREADS)
            assert list(o1) == list(o0), (name, seed)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            f.write("# Exact (l,d)-motif set of one synthetic planted instance,\n")
            f.write("# written by tests/golden/make_golden.py from the CPU oracle\n")
            f.write("# (%s).\n" % ("sample-driven O1 and brute-force O0 agree"
                                   if both else "sample-driven O1"))
            f.write("config = %s\nseed = %d\n" % (name, seed))
            f.write("n = %d\nm = %d\nl = %d\nd = %d\n"
                    % (inst.n, inst.m, inst.l, inst.d))
            f.write("input_sha256 = %s\n" % hashlib.sha256(inst.seqs).hexdigest())
            f.write("planted = %s\n" % inst.motif.decode())
            f.write("hcanon = %d\n" % h)
            f.write("count = %d\n" % len(o1))
            f.write("motifs = %s\n" % ",".join(str(int(v)) for v in o1))
            f.write("motif_strings = %s\n" % ",".join(
                oracle.decode_code(v, inst.l).decode() for v in o1))
            f.write("oracle_seconds = %.1f\n" % (t1 - t0))
        os.replace(tmp, path)
        print(name, seed, len(o1), "h=%d O1 %.1fs" % (h, t1 - t0), flush=True)


def codes_sha256(codes) -> str:
    return hashlib.sha256(codes.astype("<u8").tobytes()).hexdigest()


SET_HEADER = ("# index n m l d input_sha256 count hcanon codes_sha256 codes\n"
              "# (codes: the ascending motif codes when there are at most 64,\n"
              "# else '-'; codes_sha256 hashes all of them as little-endian\n"
              "# uint64)\n")


def _done_indices(path):
    done = set()
    if os.path.exists(path):
        for line in open(path):
            if line.strip() and not line.startswith("#") and "=" not in line:
                done.add(int(line.split()[0]))
    return done


def _append_sets(path, header, items):
    """items: (index, Instance); one line per instance, appended as each
    finishes, so that an interrupted run resumes."""
    done = _done_indices(path)
    if not os.path.exists(path):
        with open(path, "w") as f:
            f.write(header)
            f.write(SET_HEADER)
    for idx, inst in items:
        if idx in done:
            continue
        t0 = time.time()
        got, h = oracle.o1(inst.seqs, inst.n, inst.m, inst.l, inst.d,
                           threads=THREADS)
        codes = ",".join(str(int(v)) for v in got) if len(got) <= 64 else "-"
        with open(path, "a") as f:
            f.write("%d %d %d %d %d %s %d %d %s %s\n" % (
                idx, inst.n, inst.m, inst.l, inst.d,
                hashlib.sha256(inst.seqs).hexdigest(), len(got), h,
                codes_sha256(got), codes if codes else "none"))
        print(os.path.basename(path), idx, (inst.l, inst.d, inst.n, inst.m),
              len(got), "%.1fs" % (time.time() - t0), flush=True)


def main_batched():
    insts = pmsgen.batched(seed=7, count=256)
    path = os.path.join(HERE, "batched_seed7.txt")
    header = ("# Exact motif sets of the 256 instances of pmsgen.batched(seed=7),\n"
              "# written by tests/golden/make_golden.py from the CPU oracle O1.\n"
              "recipe = batched(seed=7, count=256)\n")
    # cheapest first, so a partial file already covers most instances
    order = sorted(range(len(insts)), key=lambda i: (insts[i].l, insts[i].m))
    _append_sets(path, header, [(i, insts[i]) for i in order])


# Served stream: every request with l <= 13, and a seeded sample of at least
# 10% of the (15,5), (17,6) and (19,7) requests (a (19,7) set takes about an
# hour and a half of eight cores, so that sample fills in over time).
SERVED_SAMPLE_SEED = 1511
SERVED_SAMPLE_FRAC = 0.10


def served_selection(reqs):
    import math
    import random
    sel = [r.index for r in reqs if r.inst.l <= 13]
    for ld in ((15, 5), (17, 6), (19, 7)):
        pool = [r.index for r in reqs if (r.inst.l, r.inst.d) == ld]
        k = int(math.ceil(SERVED_SAMPLE_FRAC * len(pool)))
        sel += random.Random(SERVED_SAMPLE_SEED + ld[0]).sample(pool, k)
    return sorted(sel, key=lambda i: (reqs[i].inst.l, i))


def main_served(upto_l=19):
    reqs = pmsgen.served(seed=11, count=2000)
    path = os.path.join(HERE, "served_seed11.txt")
    header = ("# Exact motif sets of the requests of pmsgen.served(seed=11,\n"
              "# count=2000) with l <= 13 and of a seeded 10%% sample of the\n"
              "# (15,5), (17,6) and (19,7) requests (random.Random(%d + l).sample),\n"
              "# written by tests/golden/make_golden.py from the CPU oracle O1.\n"
              "recipe = served(seed=11, count=2000)\n" % SERVED_SAMPLE_SEED)
    sel = [i for i in served_selection(reqs) if reqs[i].inst.l <= upto_l]
    _append_sets(path, header, [(i, reqs[i].inst) for i in sel])


# Harder instances (Table 3.3's (19,7) and (21,8) at n = 20, m = 600,
# seed 1): the motifs O1 derives from a few reference l-mers of s_1 (the
# plant's offset and seeded others). Each is a subset of the whole set.
# (O1 gives one thread per reference, so each takes minutes at (19,7) and
# a quarter of an hour at (21,8); a (23,9) reference would take hours.)
HARD = [(19, 7, 3), (21, 8, 3)]


def main_hard():
    import random
    path = os.path.join(HERE, "hard_refs_seed1.txt")
    done = set()
    if os.path.exists(path):
        for line in open(path):
            if line.strip() and not line.startswith("#"):
                t = line.split()
                done.add((int(t[0]), int(t[1]), int(t[2])))
    else:
        with open(path, "w") as f:
            f.write("# Motifs that the CPU oracle O1 derives from single reference\n"
                    "# l-mers of s_1 (offset j) of pmsgen.planted(1, 20, 600, l, d):\n"
                    "# each list is a subset of the instance's motif set.\n"
                    "# Written by tests/golden/make_golden.py.\n"
                    "# l d j input_sha256 hcanon_of_j count codes\n")
    for l, d, k in HARD:
        inst = pmsgen.planted(1, 20, 600, l, d)
        L = 600 - l + 1
        refs = [inst.positions[0]]
        others = [j for j in range(L) if j != inst.positions[0]]
        refs += random.Random(1000 + l).sample(others, k - 1)
        for j in refs:
            if (l, d, j) in done:
                continue
            t0 = time.time()
            got, h = oracle.o1(inst.seqs, 20, 600, l, d, ref_begin=j,
                               ref_end=j + 1, threads=THREADS)
            with open(path, "a") as f:
                f.write("%d %d %d %s %d %d %s\n" % (
                    l, d, j, hashlib.sha256(inst.seqs).hexdigest(), h,
                    len(got), ",".join(str(int(v)) for v in got) or "none"))
            print("hard", l, d, j, len(got), "%.1fs" % (time.time() - t0),
                  flush=True)


# Every (19,7) request of the served stream: the motifs O1 derives from two
# reference l-mers of s_1 (the plant's offset and one seeded other), each a
# subset of the request's motif set. A whole (19,7) set takes about an hour
# and a half of eight cores, a single reference about a minute of one.
def main_served_refs():
    import concurrent.futures as cf
    import random
    reqs = pmsgen.served(seed=11, count=2000)
    path = os.path.join(HERE, "served_seed11_refs.txt")
    done = set()
    if os.path.exists(path):
        for line in open(path):
            if line.strip() and not line.startswith("#"):
                t = line.split()
                done.add((int(t[0]), int(t[3])))
    else:
        with open(path, "w") as f:
            f.write("# Motifs that the CPU oracle O1 derives from single reference\n"
                    "# l-mers of s_1 (offset j) of the (19,7) requests of\n"
                    "# pmsgen.served(seed=11, count=2000): each list is a subset\n"
                    "# of the request's motif set. Written by\n"
                    "# tests/golden/make_golden.py.\n"
                    "# index l d j input_sha256 hcanon_of_j count codes\n")
    jobs = []
    for r in reqs:
        x = r.inst
        if (x.l, x.d) != (19, 7):
            continue
        L = x.m - x.l + 1
        others = [j for j in range(L) if j != x.positions[0]]
        for j in [x.positions[0],
                  random.Random(2000 + r.index).choice(others)]:
            if (r.index, j) not in done:
                jobs.append((r.index, x, j))

    def one(job):
        idx, x, j = job
        got, h = oracle.o1(x.seqs, x.n, x.m, x.l, x.d, ref_begin=j,
                           ref_end=j + 1, threads=1)
        return idx, x, j, got, h

    with cf.ThreadPoolExecutor(max_workers=int(
            os.environ.get("GOLDEN_WORKERS", "4"))) as ex:
        for idx, x, j, got, h in ex.map(one, jobs):
            with open(path, "a") as f:
                f.write("%d %d %d %d %s %d %d %s\n" % (
                    idx, x.l, x.d, j, hashlib.sha256(x.seqs).hexdigest(), h,
                    len(got), ",".join(str(int(v)) for v in got) or "none"))
            print("served refs", idx, j, len(got), flush=True)


# Long motifs: planted (40,4), n = 20, m = 600, seed 1, from W1 (the
# 128-bit-code oracle; motifs written as decimal integers).
def main_wide():
    path = os.path.join(HERE, "wide_40_4_seed1.txt")
    if os.path.exists(path):
        return
    inst = pmsgen.planted(1, 20, 600, 40, 4)
    t0 = time.time()
    got, h = oracle.o1_wide(inst.seqs, 20, 600, 40, 4, threads=THREADS)
    t1 = time.time()
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("# Exact (40,4)-motif set of one synthetic planted instance,\n")
        f.write("# written by tests/golden/make_golden.py from the CPU oracle\n")
        f.write("# (W1, sample-driven over 128-bit codes).\n")
        f.write("n = 20\nm = 600\nl = 40\nd = 4\nseed = 1\n")
        f.write("input_sha256 = %s\n" % hashlib.sha256(inst.seqs).hexdigest())
        f.write("planted = %s\n" % inst.motif.decode())
        f.write("hcanon = %d\n" % h)
        f.write("count = %d\n" % len(got))
        f.write("motifs = %s\n" % ",".join(str(v) for v in got))
        f.write("oracle_seconds = %.1f\n" % (t1 - t0))
    os.replace(tmp, path)
    print("wide 40 4", len(got), "h=%d %.1fs" % (h, t1 - t0), flush=True)


if __name__ == "__main__":
    mode = sys.argv[1] if len(sys.argv) > 1 else ""
    if mode in ("large", "batched", "served", "hard", "wide", "served_refs"):
        {"large": main_large, "batched": main_batched,
         "served": main_served, "hard": main_hard, "wide": main_wide,
         "served_refs": main_served_refs}[mode]()
        sys.exit(0)
    if len(sys.argv) > 1 and sys.argv[1] == "protein":
        main_protein()
        sys.exit(0)
    if len(sys.argv) > 1 and sys.argv[1] == "quorum":
        main_quorum()
    else:
        main()
        main_quorum()
        main_protein()
