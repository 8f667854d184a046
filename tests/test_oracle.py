"""Pins for the CPU oracle: the thesis's worked example, closed forms,
brute force on tiny inputs, textbook special cases and invariants.

Everything here runs on the CPU. The expected values come from the thesis
(cited), from mathematics written out independently in this file, or from a
pure-Python brute force that shares nothing with the C oracle.
"""
import itertools
import math
import os
import random

import numpy as np
import pytest

import oracle
import pmsgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ACGT = b"ACGT"


# ---------------------------------------------------------------------------
# independent pure-Python helpers (never used by the oracle itself)
# ---------------------------------------------------------------------------

def py_dh(a, b):
    return sum(x != y for x, y in zip(a, b))


def py_code(lmer):
    c = 0
    for ch in lmer:
        c = 4 * c + ACGT.index(ch)
    return c


def py_bruteforce(rows, l, d):
    """Definition 5 with q = n, literally: every l-mer, every string."""
    out = []
    for tup in itertools.product(range(4), repeat=l):
        M = bytes(ACGT[t] for t in tup)
        if all(any(py_dh(M, s[j:j + l]) <= d for j in range(len(s) - l + 1))
               for s in rows):
            out.append(py_code(M))
    return out


def py_hcanon(rows, l, d):
    """H_canon by literal enumeration of each B(x,d) with multiplicity."""
    L = len(rows[0]) - l + 1
    h = 0
    for j in range(L):
        x = rows[0][j:j + l]
        for tup in itertools.product(range(4), repeat=l):
            M = bytes(ACGT[t] for t in tup)
            if py_dh(M, x) > d:
                continue
            e = 0
            for s in rows[1:]:
                e += 1
                if not any(py_dh(M, s[k:k + l]) <= d for k in range(L)):
                    break
            h += e * L
    return h


def rand_rows(rng, n, m, alphabet=b"ACGT"):
    return [bytes(rng.choice(alphabet) for _ in range(m)) for _ in range(n)]


def solve(rows, l, d, which="o1"):
    n, m = len(rows), len(rows[0])
    buf = b"".join(rows)
    if which == "o1":
        return [int(v) for v in oracle.o1(buf, n, m, l, d)[0]]
    return [int(v) for v in oracle.o0(buf, n, m, l, d)]


def read_kv(path):
    kv = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = [t.strip() for t in line.split("=", 1)]
            kv[k] = v
    return kv


# ---------------------------------------------------------------------------
# worked example (Sec. 3.3.1) and encoding
# ---------------------------------------------------------------------------

def test_worked_example_groups_and_distance():
    kv = read_kv(os.path.join(GOLDEN, "worked_example.txt"))
    a, b = kv["a"].encode(), kv["b"].encode()
    rc, codes_a, _ = oracle.encode(a)
    assert rc == 0 and "".join(map(str, codes_a)) == kv["codes_a"]
    rc, codes_b, _ = oracle.encode(b)
    assert rc == 0 and "".join(map(str, codes_b)) == kv["codes_b"]

    def bits(word, l):  # group bits in string order
        return "".join(str((word >> j) & 1) for j in range(l))

    ga, gb = oracle.groups(a), oracle.groups(b)
    assert bits(ga[0], 6) == kv["group1_a"]
    assert bits(ga[1], 6) == kv["group0_a"]
    assert bits(gb[0], 6) == kv["group1_b"]
    assert bits(gb[1], 6) == kv["group0_b"]
    assert bits(ga[0] ^ gb[0], 6) == kv["xor1"]
    assert bits(ga[1] ^ gb[1], 6) == kv["xor0"]
    assert bits((ga[0] ^ gb[0]) | (ga[1] ^ gb[1]), 6) == kv["or"]
    assert oracle.hamming_groups(ga, gb) == int(kv["setbits"])
    assert oracle.hamming_naive(a, b) == int(kv["setbits"])
    assert py_dh(a, b) == int(kv["setbits"])


def test_group_distance_equals_naive_random():
    rng = random.Random(5)
    for _ in range(2000):
        l = rng.randint(1, 32)
        a = bytes(rng.choice(ACGT) for _ in range(l))
        b = bytes(rng.choice(ACGT) for _ in range(l))
        assert oracle.hamming_groups(oracle.groups(a), oracle.groups(b)) \
            == py_dh(a, b)


def test_code_is_msb_first_lexicographic():
    assert oracle.lmer_code(b"ACGT") == 0b00011011
    assert oracle.lmer_code(b"TAAA") == 3 * 64
    rng = random.Random(1)
    words = [bytes(rng.choice(ACGT) for _ in range(7)) for _ in range(300)]
    assert sorted(words) == sorted(words, key=oracle.lmer_code)
    for w in words:
        assert oracle.decode_code(oracle.lmer_code(w), 7) == w


def test_bad_bytes_rejected():
    rc, _, bad = oracle.encode(b"ACGTN")
    assert rc == oracle.OR_EBASE and bad == 4
    rc, _, bad = oracle.encode(b"acgt")
    assert rc == oracle.OR_EBASE and bad == 0
    with pytest.raises(oracle.OracleError):
        oracle.o1(b"ACGTACGTAX", 1, 10, 3, 1)
    with pytest.raises(oracle.OracleError):
        oracle.o1(b"ACGTACGTAC", 1, 10, 3, 3)   # d >= l
    with pytest.raises(oracle.OracleError):
        oracle.o1(b"ACGT", 1, 4, 5, 1)           # l > m


# ---------------------------------------------------------------------------
# sphere sizes (Table 3.1: B(a,R), n_B(l,d))
# ---------------------------------------------------------------------------

def py_ball_size(l, d, sigma):
    return sum(1 for t in itertools.product(range(sigma), repeat=l)
               if sum(v != 0 for v in t) <= d)


@pytest.mark.parametrize("l,d,sigma", [(4, 2, 2), (5, 2, 4), (6, 3, 4),
                                       (7, 1, 4), (3, 2, 4), (6, 6, 2)])
def test_nb_closed_form_vs_count(l, d, sigma):
    assert oracle.nb(l, d, sigma) == py_ball_size(l, d, sigma)


def test_nb_binary_tree_example():
    # T_2(1010) over the alphabet {0,1} (Sec. 3.2.1): root, 4 nodes at depth
    # 1, C(4,2) = 6 at depth 2.
    assert oracle.nb(4, 2, 2) == 11


@pytest.mark.parametrize("l,d,expect", [(9, 2, 352), (13, 4, 66379),
                                        (6, 5, 3367), (8, 3, 1789)])
def test_single_lmer_gives_whole_sphere(l, d, expect):
    # n = 1 and m = l: R is exactly B(s_1, d), n_B(l,d) elements.
    rng = random.Random(l * 31 + d)
    x = bytes(rng.choice(ACGT) for _ in range(l))
    got, h = oracle.o1(x, 1, l, l, d)
    assert len(got) == expect == oracle.nb(l, d)
    assert h == 0   # no other strings to examine
    assert all(py_dh(oracle.decode_code(c, l), x) <= d for c in got[:500])


# ---------------------------------------------------------------------------
# brute force on tiny inputs
# ---------------------------------------------------------------------------

def test_o1_o0_match_python_bruteforce():
    rng = random.Random(2024)
    for trial in range(40):
        l = rng.randint(1, 5)
        d = rng.randint(0, l - 1)
        n = rng.randint(1, 4)
        m = rng.randint(l, 10)
        rows = rand_rows(rng, n, m)
        want = py_bruteforce(rows, l, d)
        assert solve(rows, l, d, "o1") == want, (rows, l, d)
        assert solve(rows, l, d, "o0") == want, (rows, l, d)


def test_hcanon_matches_literal_count():
    rng = random.Random(77)
    for _ in range(15):
        l = rng.randint(2, 5)
        d = rng.randint(0, l - 1)
        n = rng.randint(1, 4)
        m = rng.randint(l, 9)
        rows = rand_rows(rng, n, m)
        _, h = oracle.o1(b"".join(rows), n, m, l, d)
        assert h == py_hcanon(rows, l, d)


def test_o0_o1_random_small():
    rng = random.Random(99)
    for _ in range(30):
        l = rng.randint(3, 8)
        d = rng.randint(0, min(3, l - 1))
        n = rng.randint(1, 6)
        m = rng.randint(l, 40)
        rows = rand_rows(rng, n, m)
        assert solve(rows, l, d, "o1") == solve(rows, l, d, "o0")


@pytest.mark.parametrize("rows,l,d", [
    ([b"AAAAAAAAAA"] * 3, 4, 1),                       # all-A
    ([b"ACACACACAC", b"CACACACACA", b"ACACACACAC"], 4, 1),  # periodic
    ([b"ACGTTGCA", b"TTGCAACG", b"GCAACGTT"], 3, 0),   # d = 0
    ([b"GATTACA"], 5, 2),                              # n = 1
    ([b"ACGTA", b"TTTTT", b"ACCTA"], 5, 2),            # m = l
    ([b"AAAAAAAA", b"CCCCCCCC"], 4, 3),               # d = l - 1
    ([b"ACGT", b"TGCA"], 1, 0),                        # l = 1
])
def test_adversarial(rows, l, d):
    want = py_bruteforce(rows, l, d) if l <= 5 else solve(rows, l, d, "o0")
    assert solve(rows, l, d, "o1") == want
    assert solve(rows, l, d, "o0") == want


def test_last_lmer_counts():
    # ACGT sits at the last offset m-l of the first string and its only
    # neighbour in the second string (ACGA) at the last offset there too
    # (Definition 2: all m-l+1 offsets count).
    rows = [b"GGGGACGT", b"TTTTACGA"]
    got = solve(rows, 4, 1)
    assert py_code(b"ACGT") in got
    assert got == py_bruteforce(rows, 4, 1)


def test_threshold_inclusive():
    # distance exactly d counts (Definition 5: "no more than d")
    rows = [b"AAAA", b"AACC"]
    got = solve(rows, 4, 1)
    assert py_code(b"AAAC") in got and py_code(b"AACA") in got
    assert py_code(b"AAAA") not in got      # distance 2 from AACC


# ---------------------------------------------------------------------------
# special cases that reduce to textbook computations
# ---------------------------------------------------------------------------

def test_d0_is_set_intersection():
    rng = random.Random(3)
    for _ in range(20):
        l = rng.randint(2, 6)
        n = rng.randint(1, 5)
        m = rng.randint(l, 30)
        rows = rand_rows(rng, n, m, alphabet=b"AC" if rng.random() < .5
                         else ACGT)
        sets = [set(py_code(s[j:j + l]) for j in range(m - l + 1))
                for s in rows]
        inter = sorted(set.intersection(*sets))
        assert solve(rows, l, 0) == inter


def pair_count(l, d, h):
    """|B(x,d) ∩ B(y,d)| for d_H(x,y) = h, by counting: on the l-h agreeing
    positions change a of them (3 letters each); on the h differing ones take
    b letters from x, c from y and e others (2 letters each)."""
    tot = 0
    for a in range(l - h + 1):
        for b in range(h + 1):
            for c in range(h - b + 1):
                e = h - b - c
                if a + (h - b) <= d and a + (h - c) <= d:
                    tot += (math.comb(l - h, a) * 3 ** a * math.factorial(h)
                            // (math.factorial(b) * math.factorial(c)
                                * math.factorial(e)) * 2 ** e)
    return tot


def test_pair_closed_form_small_table():
    # two 5-mers, radius 2: the intersection depends on their distance only
    assert [pair_count(5, 2, h) for h in range(6)] == \
        [oracle.nb(5, 2), pair_count(5, 2, 1), 34, 18, 6, 0]
    x = b"ACGTA"
    for h, y in enumerate([b"ACGTA", b"CCGTA", b"CAGTA", b"CATTA", b"CATGA",
                           b"CATGC"]):
        assert py_dh(x, y) == h
        assert len(py_bruteforce([x, y], 5, 2)) == pair_count(5, 2, h)


def test_two_lmers_closed_form():
    rng = random.Random(11)
    for _ in range(30):
        l = rng.randint(3, 9)
        d = rng.randint(0, min(4, l - 1))
        x = bytes(rng.choice(ACGT) for _ in range(l))
        y = bytes(rng.choice(ACGT) for _ in range(l))
        got = solve([x, y], l, d)
        assert len(got) == pair_count(l, d, py_dh(x, y))


# ---------------------------------------------------------------------------
# invariants on generated instances
# ---------------------------------------------------------------------------

def relabel(rows, perm):
    tab = bytes.maketrans(ACGT, bytes(ACGT[p] for p in perm))
    return [r.translate(tab) for r in rows]


def test_invariants_on_planted_instance():
    inst = pmsgen.planted(5, 8, 60, 7, 1)
    rows = inst.rows()
    l, d = inst.l, inst.d
    R = solve(rows, l, d)
    # soundness, checked by the naive scan
    for c in R:
        M = oracle.decode_code(c, l)
        assert all(any(py_dh(M, s[j:j + l]) <= d
                       for j in range(len(s) - l + 1)) for s in rows)
        assert oracle.is_motif(inst.seqs, inst.n, inst.m, l, d, c)
    # the planted motif is always recovered
    assert py_code(inst.motif) in R
    # string order does not matter
    rng = random.Random(0)
    perm_rows = rows[:]
    rng.shuffle(perm_rows)
    assert solve(perm_rows, l, d) == R
    # alphabet relabelling maps R to pi(R)
    perm = [2, 0, 3, 1]
    R2 = solve(relabel(rows, perm), l, d)
    mapped = sorted(py_code(oracle.decode_code(c, l).translate(
        bytes.maketrans(ACGT, bytes(ACGT[p] for p in perm)))) for c in R)
    assert R2 == mapped
    # reversing every string reverses every motif
    R3 = solve([r[::-1] for r in rows], l, d)
    assert R3 == sorted(py_code(oracle.decode_code(c, l)[::-1]) for c in R)
    # monotone in d, and in the set of strings
    Rd1 = solve(rows, l, d + 1)
    assert set(R) <= set(Rd1)
    Rmore = solve(rows + [b"ACGT" * 15], l, d)
    assert set(Rmore) <= set(R)


def py_is_motif(rows, l, d, M):
    """Definition 5 for one l-mer M, literally: every string has an l-mer
    within distance d of M."""
    return all(any(py_dh(M, s[j:j + l]) <= d for j in range(len(s) - l + 1))
               for s in rows)


def test_is_motif_every_code_tiny():
    # the per-code check accepts exactly the codes of Definition 5, over the
    # whole code space: members and non-members alike
    rng = random.Random(21)
    n_false = n_true = 0
    for _ in range(25):
        l = rng.randint(2, 5)
        d = rng.randint(0, min(2, l - 1))
        n = rng.randint(1, 4)
        m = rng.randint(l, 12)
        rows = rand_rows(rng, n, m)
        buf = b"".join(rows)
        for c in range(4 ** l):
            want = py_is_motif(rows, l, d, oracle.decode_code(c, l))
            assert oracle.is_motif(buf, n, m, l, d, c) == want, (rows, l, d, c)
            n_true += want
            n_false += not want
    assert n_true > 200 and n_false > 2000


def test_is_motif_rejects_distance_d_plus_1():
    # a code within d of an l-mer in every string but one, where its nearest
    # l-mer is at exactly d + 1, is not a motif; moving one base of that
    # l-mer onto the code makes it one
    l, d = 6, 2
    M = b"ACGTAC"
    near = b"ACGTTT"                      # distance 2 = d
    far = b"GTGTTC"                       # distance 3 = d + 1
    assert py_dh(M, near) == d and py_dh(M, far) == d + 1
    rows = [b"CC" + near + b"CC", b"GG" + M + b"GG", b"AA" + far + b"AA"]
    # no other window of the last string is within d (checked literally)
    assert not py_is_motif(rows, l, d, M)
    buf = b"".join(rows)
    code = py_code(M)
    assert oracle.is_motif(buf, 3, 10, l, d, code) is False
    assert oracle.hit_count(buf, 3, 10, l, d, code) == 2
    fixed = rows[:2] + [b"AA" + b"ACGTTC" + b"AA"]   # distance 1 now
    assert py_is_motif(fixed, l, d, M)
    assert oracle.is_motif(b"".join(fixed), 3, 10, l, d, code) is True


def test_is_motif_last_string_and_last_offset():
    # the only string without a neighbour is the last one; the only
    # neighbour of another string sits at its last offset
    l, d = 5, 1
    M = b"GATTC"
    rows = [b"TTTT" + M, b"CCCCCCCCC", b"AAAA" + b"GATTA"]
    assert not py_is_motif(rows, l, d, M)
    buf = b"".join(rows)
    assert oracle.is_motif(buf, 3, 9, l, d, py_code(M)) is False
    rows2 = [b"TTTT" + M, b"CCCC" + b"GCTTC", b"AAAA" + b"GATTA"]
    assert py_is_motif(rows2, l, d, M)
    assert oracle.is_motif(b"".join(rows2), 3, 9, l, d, py_code(M)) is True


def test_is_motif_planted_members_and_non_members():
    # full-size (9,2) instance: the check agrees with membership in the
    # stored set (pinned above through O0) on members and on sampled
    # non-members, and non-members miss at least one string
    kv, motifs = load_golden("pms_9_2_seed1.txt")
    inst = pmsgen.plain("pms_9_2", 1)
    n, m, l, d = inst.n, inst.m, inst.l, inst.d
    member = set(motifs)
    for c in motifs:
        assert oracle.is_motif(inst.seqs, n, m, l, d, c)
    rng = random.Random(92)
    rows = inst.rows()
    sample = [rng.randrange(4 ** l) for _ in range(300)]
    # codes one base away from a member are near misses
    for c in motifs:
        for p in range(l):
            sample.append(c ^ (1 << (2 * p)))
    for c in sample:
        got = oracle.is_motif(inst.seqs, n, m, l, d, c)
        assert got == (c in member), c
        if not got:
            assert oracle.hit_count(inst.seqs, n, m, l, d, c) < n
    # a literal recheck of a few rejected near misses
    for c in [x for x in sample[300:] if x not in member][:6]:
        assert not py_is_motif(rows, l, d, oracle.decode_code(c, l))


def test_planted_generator_rule():
    for seed in range(5):
        inst = pmsgen.planted(seed, 12, 80, 9, 3)
        for i, row in enumerate(inst.rows()):
            p = inst.positions[i]
            assert 0 <= p <= inst.m - inst.l
            occ = row[p:p + inst.l]
            assert py_dh(occ, inst.motif) == inst.d
            assert sorted(j for j in range(inst.l)
                          if occ[j] != inst.motif[j]) == sorted(inst.mutated[i])


def test_generator_streams():
    import ctypes
    lib = pmsgen._load()
    x = ctypes.c_uint64(0)
    # SplitMix64 from state 0 (published first outputs)
    assert lib.pmsgen_splitmix64(ctypes.byref(x)) == 0xE220A8397B1DCDAF
    assert lib.pmsgen_splitmix64(ctypes.byref(x)) == 0x6E789E6AA1B965F4
    for seed in (0, 1, 12345, 2**63 + 5):
        a, b = pmsgen.Rng(seed), pmsgen.PyRng(seed)
        assert [a.next() for _ in range(50)] == [b.next() for _ in range(50)]
    assert pmsgen.planted(3, 4, 50, 8, 2).seqs == \
        pmsgen.planted(3, 4, 50, 8, 2).seqs


def test_hcanon_bounds_and_per_reference():
    inst = pmsgen.planted(9, 6, 50, 7, 2)
    L = inst.m - inst.l + 1
    R, h, per = oracle.o1(inst.seqs, inst.n, inst.m, 7, 2, per_ref=True)
    assert int(per.sum()) == h
    cand = L * oracle.nb(7, 2)
    assert cand * L <= h <= cand * L * (inst.n - 1)
    # a partial range of references sees exactly its share
    _, h2, per2 = oracle.o1(inst.seqs, inst.n, inst.m, 7, 2, ref_begin=10,
                            ref_end=20, per_ref=True)
    assert h2 == int(per[10:20].sum()) and (per2 == per[10:20]).all()


def test_thread_count_does_not_change_result():
    inst = pmsgen.planted(2, 10, 120, 8, 2)
    a = oracle.o1(inst.seqs, 10, 120, 8, 2, threads=1)
    b = oracle.o1(inst.seqs, 10, 120, 8, 2, threads=7)
    assert (a[0] == b[0]).all() and a[1] == b[1]
    assert (oracle.o0(inst.seqs, 10, 120, 8, 2, threads=1)
            == oracle.o0(inst.seqs, 10, 120, 8, 2, threads=5)).all()


# ---------------------------------------------------------------------------
# stored results at the full (9,2) and (13,4) sizes
# ---------------------------------------------------------------------------

def load_golden(name):
    path = os.path.join(GOLDEN, name)
    kv = read_kv(path)
    motifs = [int(x) for x in kv["motifs"].split(",")] if kv["motifs"] else []
    return kv, motifs


@pytest.mark.parametrize("name,seed", [("pms_9_2", k) for k in range(1, 6)] +
                         [("pms_13_4", k) for k in range(1, 6)])
def test_golden_full_size(name, seed):
    kv, motifs = load_golden("%s_seed%d.txt" % (name, seed))
    inst = pmsgen.plain(name, seed)
    import hashlib
    assert hashlib.sha256(inst.seqs).hexdigest() == kv["input_sha256"], \
        "generator stream changed; regenerate the golden files"
    got, h = oracle.o1(inst.seqs, inst.n, inst.m, inst.l, inst.d)
    assert [int(v) for v in got] == motifs
    assert h == int(kv["hcanon"])
    assert py_code(inst.motif) in motifs


@pytest.mark.parametrize("seed", range(1, 6))
def test_golden_17_6_stored(seed):
    # the stored (17,6) sets (O1 over all 584 references, minutes of CPU
    # each) belong to the generator's current stream, hold the plant, and
    # every stored code is a motif by the direct check of Definition 5;
    # PMS_SLOW=1 recomputes them whole
    import hashlib
    kv, motifs = load_golden("pms_17_6_seed%d.txt" % seed)
    inst = pmsgen.plain("pms_17_6", seed)
    assert hashlib.sha256(inst.seqs).hexdigest() == kv["input_sha256"]
    assert int(kv["count"]) == len(motifs) and motifs == sorted(set(motifs))
    assert py_code(inst.motif) in motifs
    for c in motifs:
        assert oracle.is_motif(inst.seqs, inst.n, inst.m, inst.l, inst.d, c)
    assert int(kv["hcanon"]) > 5e12


@pytest.mark.slow
@pytest.mark.parametrize("seed", range(1, 6))
def test_golden_17_6_recompute(seed):
    kv, motifs = load_golden("pms_17_6_seed%d.txt" % seed)
    inst = pmsgen.plain("pms_17_6", seed)
    got, h = oracle.o1(inst.seqs, inst.n, inst.m, inst.l, inst.d)
    assert [int(v) for v in got] == motifs
    assert h == int(kv["hcanon"])
