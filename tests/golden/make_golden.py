"""Write the stored full-size results used by tests/test_oracle.py.

Calls only the CPU oracle (both O1 and the brute force O0, which must agree)
on inputs from the seeded generator; nothing here touches the GPU library.
Run from the repository root:  python tests/golden/make_golden.py
(add "quorum" or "protein" to write only those files)
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


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "protein":
        main_protein()
        sys.exit(0)
    if len(sys.argv) > 1 and sys.argv[1] == "quorum":
        main_quorum()
    else:
        main()
        main_quorum()
        main_protein()
