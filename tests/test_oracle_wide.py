"""Pins of the long-motif oracle W1 (1 <= l <= 64, 128-bit codes).

Sec. 3.3.1 keeps an l-mer that does not fit one machine word in ceil(l/32)
words per group; the problem itself (Definition 5) does not change with l.
W1 is pinned to:
- the already pinned O1 wherever both apply (l <= 32): same set, same
  H_canon;
- Definition 5 written as the intersection over strings of the unions of
  the d-spheres of their l-mers, in pure Python on Python integers, for
  l from 33 to 64;
- closed forms and special cases: one string of length l gives exactly
  n_B(l,d) motifs (Table 3.1), d = 0 gives the intersection of the strings'
  l-mer sets;
- a literal count of H_canon;
- its per-code check, on members and non-members.
"""
import itertools
import math
import random

import pytest

import oracle
import pmsgen

ACGT = b"ACGT"


def code_of(s: bytes) -> int:
    c = 0
    for ch in s:
        c = 4 * c + ACGT.index(ch)
    return c


def sphere(y: bytes, d: int):
    """Codes of B(y, d): every string within Hamming distance d of y."""
    l = len(y)
    base = code_of(y)
    out = set()
    for k in range(d + 1):
        for pos in itertools.combinations(range(l), k):
            for deltas in itertools.product((1, 2, 3), repeat=k):
                c = base
                for p, dl in zip(pos, deltas):
                    c ^= dl << (2 * (l - 1 - p))
                out.add(c)
    return out


def definition5(seqs: bytes, n, m, l, d):
    """Intersection over the strings of the union of the d-spheres of
    their l-mers."""
    res = None
    for i in range(n):
        s = seqs[i * m:(i + 1) * m]
        u = set()
        for j in range(m - l + 1):
            u |= sphere(s[j:j + l], d)
        res = u if res is None else (res & u)
    return sorted(res)


def mutated_family(rng, n, m, l, changes, keep=None):
    """n strings of length m: copies of one random string, each with a few
    random substitutions (none inside the window keep = (start, end)), so
    that the strings share many neighbourhoods."""
    base = bytes(rng.choice(ACGT) for _ in range(m))
    free = [p for p in range(m) if keep is None or not keep[0] <= p < keep[1]]
    rows = []
    for _ in range(n):
        r = bytearray(base)
        for p in rng.sample(free, changes):
            r[p] = rng.choice([b for b in ACGT if b != r[p]])
        rows.append(bytes(r))
    return b"".join(rows)


def test_wide_equals_o1_where_both_apply():
    rng = random.Random(4101)
    for t in range(30):
        l = rng.choice([3, 5, 8, 11, 16, 32])
        d = rng.randint(0, min(3, l - 1))
        n = rng.randint(1, 4)
        m = l + rng.randint(0, 12)
        seqs = bytes(rng.choice(ACGT) for _ in range(n * m))
        if t % 3 == 0 and n > 1:
            seqs = mutated_family(rng, n, m, l, 2)
        if l == 32 and d > 2:
            d = 2
        want, hw = oracle.o1(seqs, n, m, l, d)
        got, hg = oracle.o1_wide(seqs, n, m, l, d)
        assert got == [int(v) for v in want], (t, n, m, l, d)
        assert hg == hw, (t, n, m, l, d)


@pytest.mark.parametrize("l,d,n,extra,changes,seed,size", [
    (33, 1, 3, 4, 1, 1, 8), (33, 2, 2, 3, 2, 2, 24), (36, 2, 3, 2, 2, 3, 15),
    (40, 2, 2, 4, 2, 5, 30), (48, 1, 4, 3, 1, 6, 4), (57, 2, 2, 2, 2, 7, 18),
    (64, 1, 3, 3, 1, 8, 4), (64, 2, 2, 2, 2, 9, 1164),
    (40, 1, 3, 3, 4, 10, 0),
])
def test_wide_equals_definition5(l, d, n, extra, changes, seed, size):
    rng = random.Random(seed)
    m = l + extra
    seqs = mutated_family(rng, n, m, l, changes)
    want = definition5(seqs, n, m, l, d)
    got, _ = oracle.o1_wide(seqs, n, m, l, d)
    assert got == want
    # the sizes were read off this definition once; they keep the cases
    # from drifting into empty or trivial sets
    assert len(want) == size


def test_wide_planted_instances():
    for seed, (l, d) in enumerate([(35, 2), (40, 3), (64, 3)]):
        inst = pmsgen.planted(seed + 1, 4, 90, l, d)
        got, _ = oracle.o1_wide(inst.seqs, 4, 90, l, d)
        assert code_of(inst.motif) in got
        for c in got:
            assert oracle.is_motif_wide(inst.seqs, 4, 90, l, d, c)


@pytest.mark.parametrize("l,d", [(33, 2), (40, 2), (64, 1), (50, 3)])
def test_wide_one_string_gives_the_sphere(l, d):
    rng = random.Random(l * 7 + d)
    s = bytes(rng.choice(ACGT) for _ in range(l))
    got, h = oracle.o1_wide(s, 1, l, l, d)
    nb = sum(math.comb(l, k) * 3 ** k for k in range(d + 1))
    assert len(got) == nb
    assert h == 0                 # no other string to test
    if nb <= 20000:
        assert got == sorted(sphere(s, d))


def test_wide_d0_is_the_lmer_intersection():
    rng = random.Random(77)
    for l, n, m in [(33, 3, 45), (40, 2, 60), (64, 3, 70)]:
        # a protected window keeps one l-mer common to every string
        seqs = mutated_family(rng, n, m, l, 3, keep=(m - l, m))
        sets = []
        for i in range(n):
            s = seqs[i * m:(i + 1) * m]
            sets.append({code_of(s[j:j + l]) for j in range(m - l + 1)})
        want = sorted(set.intersection(*sets))
        got, _ = oracle.o1_wide(seqs, n, m, l, 0)
        assert got == want and want


def hcanon_literal(seqs, n, m, l, d):
    """For every candidate of every sphere B(x,d), x an l-mer of s_1 (with
    multiplicity), L times the strings s_2.. examined up to the first one
    without an l-mer within d."""
    L = m - l + 1
    rows = [seqs[i * m:(i + 1) * m] for i in range(n)]
    lm = [[code_of(r[j:j + l]) for j in range(L)] for r in rows]

    def dist(a, b):
        return sum(1 for p in range(l)
                   if ((a >> (2 * p)) & 3) != ((b >> (2 * p)) & 3))

    total = 0
    for j in range(L):
        for c in sphere(rows[0][j:j + l], d):
            for i in range(1, n):
                total += L
                if min(dist(c, y) for y in lm[i]) > d:
                    break
    return total


def test_wide_hcanon_literal():
    rng = random.Random(5)
    for l, d, n, m in [(33, 1, 3, 36), (34, 2, 3, 36), (40, 1, 4, 42)]:
        seqs = mutated_family(rng, n, m, l, 3)
        _, h = oracle.o1_wide(seqs, n, m, l, d)
        assert h == hcanon_literal(seqs, n, m, l, d)


def test_is_motif_wide_both_branches():
    rng = random.Random(11)
    l, d, n, m = 40, 2, 3, 46
    seqs = mutated_family(rng, n, m, l, 3)
    rows = [seqs[i * m:(i + 1) * m] for i in range(n)]

    def literal(c):
        M = [(c >> (2 * (l - 1 - p))) & 3 for p in range(l)]
        for r in rows:
            best = min(sum(1 for p in range(l)
                           if ACGT.index(r[j + p]) != M[p])
                       for j in range(m - l + 1))
            if best > d:
                return False
        return True

    got, _ = oracle.o1_wide(seqs, n, m, l, d)
    for c in got:
        assert oracle.is_motif_wide(seqs, n, m, l, d, c)
    # a motif moved to distance d + 1 from the nearest l-mer of one string
    # is rejected exactly when that is so by the literal definition
    checked_false = 0
    for c in got[:50]:
        for p in range(l):
            c2 = c ^ (1 << (2 * p))
            want = literal(c2)
            assert oracle.is_motif_wide(seqs, n, m, l, d, c2) == want
            checked_false += not want
    assert checked_false > 0
    for _ in range(200):
        c = rng.getrandbits(2 * l)
        assert oracle.is_motif_wide(seqs, n, m, l, d, c) == literal(c)
    # codes with bits above 2l are not l-mers
    with pytest.raises(oracle.OracleError):
        oracle.is_motif_wide(seqs, n, m, l, d, 1 << (2 * l))


def test_wide_argument_checks():
    s = b"A" * 70
    for (n, m, l, d) in [(1, 70, 65, 1), (1, 70, 0, 0), (1, 30, 40, 1),
                         (1, 70, 40, 40)]:
        with pytest.raises(oracle.OracleError):
            oracle.o1_wide(s[:n * m], n, m, l, d)
    with pytest.raises(oracle.OracleError):
        oracle.o1_wide(b"ACGTN" * 8, 1, 40, 33, 1)
