"""GPU parity for the pair-based path (PMS_PATH_PAIR, Observation 3.3).

The set must equal the sample-driven oracle's (and, at (17,6), the tiled
path's) code for code, and the device's work counters must equal the
pair-based oracle's: the number of candidates (the sum over compatible
pairs of |B(x,d) ∩ B(y,d)|) and the number of compatible pairs, recounted
here. Integer results: the tolerance is zero.
"""
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
    c = pms.Context(path=pms.PATH_PAIR)
    yield c
    c.close()


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
