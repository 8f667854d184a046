"""GPU parity for the pair-based path (PMS_PATH_PAIR, Observation 3.3).

The set must equal the sample-driven oracle's (and, at (17,6), the tiled
path's) code for code. With s_2 as every l-mer's partner the device's
work counters must equal the pair-based oracle's: the number of candidates
(the sum over compatible pairs of |B(x,d) ∩ B(y,d)|) and the number of
compatible pairs, recounted here. With TraverStringRef's string reordering
(every l-mer x of s_1 paired with the string whose nearest l-mer is
farthest from x, Sec. 3.2.3; the default) the counters must equal a
recount here from literal distances and the closed-form intersection size.
Integer results: the tolerance is zero.
"""
import math
import random
import sys

import numpy as np
import pytest

import oracle
import paper_2403_00306_amd as pms
import pmsgen

pytestmark = pytest.mark.gpu

ACGT = b"ACGT"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pctx():
    c = pms.Context(path=pms.PATH_PAIR, pair_partner=1)
    yield c
    c.close()


@pytest.fixture(scope="module")
def xctx():
    c = pms.Context(path=pms.PATH_PAIR)      # partner per l-mer of s_1
    yield c
    c.close()


def inter_size(l, d, h):
    """|B(x,d) ∩ B(y,d)| for d_H(x,y) = h: on the l-h agreeing positions
    change a (3 letters each); on the h differing ones take b letters from
    x, c from y and the rest from the 2 others."""
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


def reordered_counts(seqs, n, m, l, d):
    """(pairs, candidates) when every l-mer x of s_1 pairs with the l-mers
    of the string (other than s_1) whose nearest l-mer is farthest from x,
    the lowest-numbered such string on ties."""
    rows = [seqs[i * m:(i + 1) * m] for i in range(n)]
    L = m - l + 1
    pairs = cand = 0
    for j in range(L):
        x = rows[0][j:j + l]
        best, part = -1, 1
        for i in range(1, n):
            md = min(py_dh(x, rows[i][k:k + l]) for k in range(L))
            if md > best:
                best, part = md, i
        for k in range(L):
            h = py_dh(x, rows[part][k:k + l])
            if h <= 2 * d:
                c = inter_size(l, d, h)
                if c:
                    pairs += 1
                    cand += c
    return pairs, cand


def py_dh(a, b):
    return sum(x != y for x, y in zip(a, b))


def compatible_pairs(seqs, m, l, d):
    s1, s2 = seqs[:m], seqs[m:2 * m]
    L = m - l + 1
    return sum(py_dh(s1[j:j + l], s2[k:k + l]) <= 2 * d
               for j in range(L) for k in range(L))


def test_pair_random_small(pctx):
    rng = random.Random(21)
    for case in range(25):
        l = rng.randint(3, 10)
        d = rng.randint(0, min(3, l - 1))
        n = rng.randint(2, 8)
        m = rng.randint(l, 60)
        seqs = bytes(rng.choice(ACGT) for _ in range(n * m))
        say("pair case", case, (n, m, l, d))
        got = pctx.solve(seqs, n, m, l, d)
        want, _ = oracle.o1(seqs, n, m, l, d)
        assert got.shape == want.shape and (got == want).all(), \
            (n, m, l, d)
        st = pctx.stats()
        _, nc = oracle.p1(seqs, n, m, l, d)
        assert st["candidates"] == nc
        assert st["pairs"] == compatible_pairs(seqs, m, l, d)


@pytest.mark.parametrize("name,seed", [("pms_9_2", 1), ("pms_9_2", 2),
                                       ("pms_13_4", 1)])
def test_pair_full_size(pctx, name, seed):
    inst = pmsgen.plain(name, seed)
    say("pair", name, seed)
    got = pctx.solve(inst.seqs, inst.n, inst.m, inst.l, inst.d)
    want, _ = oracle.o1(inst.seqs, inst.n, inst.m, inst.l, inst.d)
    assert (got == want).all()
    _, nc = oracle.p1(inst.seqs, inst.n, inst.m, inst.l, inst.d)
    assert pctx.stats()["candidates"] == nc


def test_pair_17_6_equals_tiled(pctx):
    inst = pmsgen.plain("pms_17_6", 1)
    got = pctx.solve(inst.seqs, 20, 600, 17, 6)
    st = pctx.stats()
    with pms.Context(path=pms.PATH_TILED) as c:
        want = c.solve(inst.seqs, 20, 600, 17, 6)
    assert (got == want).all()
    say("(17,6) pairs", st["pairs"], "candidates", st["candidates"],
        "ms", st["ms_main"])
    # fewer candidates than the spheres of every l-mer of s_1
    assert st["candidates"] < 584 * oracle.nb(17, 6)


def test_pair_long_motifs(pctx):
    # l up to 32 (a full 32-bit word per bit plane), planted and on
    # near-copies of one random string (one base redrawn per string), whose
    # sets are dense
    for (n, m, l, d) in [(4, 60, 32, 2), (5, 80, 20, 3), (3, 50, 25, 1)]:
        rng = random.Random(l + d)
        base = bytes(rng.choice(ACGT) for _ in range(m))
        near = bytearray()
        for _ in range(n):
            s = bytearray(base)
            s[rng.randrange(m)] = rng.choice(ACGT)
            near += s
        for kind, seqs in (("planted", pmsgen.planted(l * 7 + d, n, m, l,
                                                       d).seqs),
                           ("near-copies", bytes(near))):
            say("pair long", kind, (n, m, l, d))
            got = pctx.solve(seqs, n, m, l, d)
            want, _ = oracle.o1(seqs, n, m, l, d)
            assert got.shape == want.shape and (got == want).all(), \
                (kind, l, d)
            _, nc = oracle.p1(seqs, n, m, l, d)
            assert pctx.stats()["candidates"] == nc


def test_pair_repeats(pctx):
    # every pair compatible, every motif reached from many pairs
    rows = [b"A" * 24, b"A" * 12 + b"C" * 12, b"A" * 24]
    seqs = b"".join(rows)
    for l, d in [(4, 1), (6, 2)]:
        got = pctx.solve(seqs, 3, 24, l, d)
        want, _ = oracle.o1(seqs, 3, 24, l, d)
        assert (got == want).all()


def test_pair_string_reordering_small(xctx):
    rng = random.Random(57)
    for case in range(25):
        l = rng.randint(3, 10)
        d = rng.randint(0, min(3, l - 1))
        n = rng.randint(2, 8)
        m = rng.randint(l, 50)
        seqs = bytes(rng.choice(ACGT) for _ in range(n * m))
        say("pair reordered case", case, (n, m, l, d))
        got = xctx.solve(seqs, n, m, l, d)
        want, _ = oracle.o1(seqs, n, m, l, d)
        assert got.shape == want.shape and (got == want).all(), \
            (n, m, l, d)
        st = xctx.stats()
        assert (st["pairs"], st["candidates"]) == \
            reordered_counts(seqs, n, m, l, d), (n, m, l, d)


@pytest.mark.parametrize("name,seed", [("pms_9_2", 1), ("pms_13_4", 1)])
def test_pair_string_reordering_full_size(xctx, name, seed):
    inst = pmsgen.plain(name, seed)
    got = xctx.solve(inst.seqs, inst.n, inst.m, inst.l, inst.d)
    want, _ = oracle.o1(inst.seqs, inst.n, inst.m, inst.l, inst.d)
    assert (got == want).all()


def test_pair_string_reordering_17_6(xctx, pctx):
    # fewer candidates and Hamming tests than with s_2 as every partner,
    # the same set as the tiled path
    inst = pmsgen.plain("pms_17_6", 1)
    got = xctx.solve(inst.seqs, 20, 600, 17, 6)
    sx = xctx.stats()
    base = pctx.solve(inst.seqs, 20, 600, 17, 6)
    s2 = pctx.stats()
    with pms.Context(path=pms.PATH_TILED) as c:
        want = c.solve(inst.seqs, 20, 600, 17, 6)
    assert (got == want).all() and (base == want).all()
    say("(17,6) reordered: pairs", sx["pairs"], "candidates",
        sx["candidates"], "tests", sx["filter_tests"], "ms", sx["ms_main"],
        "| s_2: candidates", s2["candidates"], "tests", s2["filter_tests"],
        "ms", s2["ms_main"])
    assert sx["candidates"] < s2["candidates"]
    assert sx["filter_tests"] < s2["filter_tests"]


def test_pair_rejects(pctx):
    inst = pmsgen.plain("pms_9_2", 1)
    with pytest.raises(pms.PmsError):
        pctx.solve(inst.seqs[:600], 1, 600, 9, 2)          # needs n >= 2
    seqs = bytes(random.Random(2).choice(ACGT) for _ in range(3 * 40))
    with pytest.raises(pms.PmsError):
        pctx.solve(seqs, 3, 40, 25, 11)                     # 2d > 20
    with pytest.raises(pms.PmsError):
        pctx.solve_quorum(inst.seqs, 20, 600, 9, 2, 10)     # quorum: tiled
    bad = bytearray(inst.seqs)
    bad[3 * 600 + 5] = ord("x")
    with pytest.raises(pms.PmsError):
        pctx.solve(bytes(bad), 20, 600, 9, 2)
    assert len(pctx.solve(inst.seqs, 20, 600, 9, 2)) > 0
