"""Pins for the quorum oracle: (l,d,q)-motifs (Definition 5, qPMS definition).

Runs on the CPU. Expected values come from a literal pure-Python reading of
Definition 5, from a closed-form count written out here, from the already
pinned q = n oracle, or from invariants the definition implies. Nothing here
uses the GPU library.
"""
import hashlib
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


def py_dh(a, b):
    return sum(x != y for x, y in zip(a, b))


def py_code(lmer):
    c = 0
    for ch in lmer:
        c = 4 * c + ACGT.index(ch)
    return c


def py_quorum(rows, l, d, q):
    """Definition 5, literally: every l-mer M, kept when at least q strings
    have an l-mer within distance d of M."""
    out = []
    for tup in itertools.product(range(4), repeat=l):
        M = bytes(ACGT[t] for t in tup)
        hits = sum(any(py_dh(M, s[j:j + l]) <= d
                       for j in range(len(s) - l + 1)) for s in rows)
        if hits >= q:
            out.append(py_code(M))
    return out


def rand_rows(rng, n, m):
    return [bytes(rng.choice(ACGT) for _ in range(m)) for _ in range(n)]


def test_tiny_instances_match_definition():
    rng = random.Random(2024)
    for _ in range(40):
        l = rng.randint(2, 5)
        d = rng.randint(0, l - 1)
        n = rng.randint(1, 5)
        m = rng.randint(l, l + 5)
        q = rng.randint(1, n)
        rows = rand_rows(rng, n, m)
        seqs = b"".join(rows)
        want = py_quorum(rows, l, d, q)
        assert [int(v) for v in oracle.q1(seqs, n, m, l, d, q)] == want, \
            (n, m, l, d, q)
        assert [int(v) for v in oracle.q0(seqs, n, m, l, d, q)] == want


def test_q_equal_n_is_plain_pms():
    # the q = n oracle is pinned separately (test_oracle.py)
    rng = random.Random(7)
    for _ in range(12):
        l = rng.randint(4, 7)
        d = rng.randint(0, 2)
        n = rng.randint(2, 8)
        m = rng.randint(l, 40)
        seqs = b"".join(rand_rows(rng, n, m))
        pms, _ = oracle.o1(seqs, n, m, l, d)
        assert (oracle.q1(seqs, n, m, l, d, n) == pms).all()
        assert (oracle.q0(seqs, n, m, l, d, n) == pms).all()


def pair_intersection(l, d, D):
    """|B(x,d) ∩ B(y,d)| for two l-mers at distance D, counted by cases: on
    the D positions where x and y differ, M takes x's letter (a of them),
    y's letter (b) or one of the 2 others (c); on the l-D positions where
    they agree, M changes e of them (3 letters each)."""
    tot = 0
    for a in range(D + 1):
        for b in range(D + 1 - a):
            c = D - a - b
            ways = math.factorial(D) // (math.factorial(a) * math.factorial(b)
                                         * math.factorial(c))
            for e in range(l - D + 1):
                if b + c + e <= d and a + c + e <= d:
                    tot += ways * 2 ** c * math.comb(l - D, e) * 3 ** e
    return tot


@pytest.mark.parametrize("l,d", [(5, 2), (6, 2), (6, 3)])
def test_two_lmers_union_and_intersection(l, d):
    # n = 2 strings of one l-mer each: q = 1 is the union of the two
    # spheres, q = 2 their intersection
    rng = random.Random(l * 10 + d)
    nb = oracle.nb(l, d)
    for D in range(0, l + 1):
        x = bytes(rng.choice(ACGT) for _ in range(l))
        y = bytearray(x)
        for p in rng.sample(range(l), D):
            y[p] = rng.choice([c for c in ACGT if c != x[p]])
        seqs = x + bytes(y)
        inter = pair_intersection(l, d, D)
        assert len(oracle.q1(seqs, 2, l, l, d, 2)) == inter
        assert len(oracle.q1(seqs, 2, l, l, d, 1)) == 2 * nb - inter
        assert len(oracle.q0(seqs, 2, l, l, d, 1)) == 2 * nb - inter


def test_pair_intersection_formula_against_enumeration():
    # the closed form itself, against a literal count at l = 5, d = 2
    for D in range(6):
        x = b"ACGTA"
        y = bytearray(x)
        for p in range(D):
            y[p] = ACGT[(ACGT.index(x[p]) + 1) % 4]
        cnt = 0
        for tup in itertools.product(range(4), repeat=5):
            M = bytes(ACGT[t] for t in tup)
            cnt += py_dh(M, x) <= 2 and py_dh(M, y) <= 2
        assert cnt == pair_intersection(5, 2, D)


def test_monotone_in_q_and_planted_motif():
    inst = pmsgen.plain("pms_9_2", 2)
    prev = None
    for q in range(inst.n, 0, -3):
        cur = oracle.q1(inst.seqs, inst.n, inst.m, inst.l, inst.d, q)
        assert py_code(inst.motif) in set(int(v) for v in cur)
        if prev is not None:
            assert set(prev.tolist()) <= set(cur.tolist())
        prev = cur


def test_string_order_does_not_matter():
    # the reference strings of Observation 3.1 are s_1..s_{n-q+1}: a wrong
    # range or a q = n shortcut shows up as a dependence on string order
    inst = pmsgen.plain("pms_9_2", 3)
    rows = [inst.seqs[i * inst.m:(i + 1) * inst.m] for i in range(inst.n)]
    rng = random.Random(5)
    perm = list(range(inst.n))
    rng.shuffle(perm)
    shuffled = b"".join(rows[i] for i in perm)
    for q in (3, 11, 17):
        a = oracle.q1(inst.seqs, inst.n, inst.m, inst.l, inst.d, q)
        b = oracle.q1(shuffled, inst.n, inst.m, inst.l, inst.d, q)
        assert (a == b).all()


def test_hit_counts_agree_with_membership():
    inst = pmsgen.plain("pms_9_2", 1)
    q = 12
    got = set(int(v) for v in
              oracle.q1(inst.seqs, inst.n, inst.m, inst.l, inst.d, q))
    rng = random.Random(9)
    for code in rng.sample(range(4 ** inst.l), 300):
        h = oracle.hit_count(inst.seqs, inst.n, inst.m, inst.l, inst.d, code)
        assert (h >= q) == (code in got)


def test_rejects_bad_quorum():
    inst = pmsgen.plain("pms_9_2", 1)
    for q in (0, inst.n + 1):
        with pytest.raises(oracle.OracleError):
            oracle.q1(inst.seqs, inst.n, inst.m, inst.l, inst.d, q)


def read_kv(path):
    kv = {}
    for line in open(path):
        if line.startswith("#") or "=" not in line:
            continue
        k, v = line.split("=", 1)
        kv[k.strip()] = v.strip()
    return kv


@pytest.mark.parametrize("name,seed,q", [("pms_9_2", 1, 10),
                                         ("pms_9_2", 1, 15),
                                         ("pms_9_2", 2, 5)])
def test_golden_quorum(name, seed, q):
    kv = read_kv(os.path.join(GOLDEN, "%s_seed%d_q%d.txt" % (name, seed, q)))
    inst = pmsgen.plain(name, seed)
    assert hashlib.sha256(inst.seqs).hexdigest() == kv["input_sha256"]
    got = oracle.q1(inst.seqs, inst.n, inst.m, inst.l, inst.d, q)
    assert len(got) == int(kv["count"])
    assert hashlib.sha256(got.astype("<u8").tobytes()).hexdigest() == \
        kv["codes_sha256"]
