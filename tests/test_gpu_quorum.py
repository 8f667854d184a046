"""GPU parity for quorum motifs ((l,d,q)-motifs, Definition 5, q < n).

The HIP library's pms_solve_quorum against the CPU oracle (Q1, Observation
3.1), element by element on the same seeded inputs: full (9,2) instances at
several q, random small instances with ragged sizes, and the edge cases of
the quorum. At (13,4) and (17,6) with q = 10 the sets are too large for the
oracle to recompute whole, so every sampled reported code, a sample of codes
not reported, the plant, sortedness and monotonicity in q are checked
instead. Integer results: the tolerance is zero.
"""
import hashlib
import os
import random
import sys

import numpy as np
import pytest

import oracle
import paper_2403_00306_amd as pms
import pmsgen

pytestmark = pytest.mark.gpu

ACGT = b"ACGT"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = pms.Context()
    yield c
    c.close()


def code_of(lmer: bytes) -> int:
    c = 0
    for ch in lmer:
        c = 4 * c + ACGT.index(ch)
    return c


@pytest.mark.parametrize("seed,q", [(1, 1), (1, 7), (1, 19), (2, 10),
                                    (2, 16), (3, 4), (3, 12)])
def test_quorum_full_9_2(ctx, seed, q):
    inst = pmsgen.plain("pms_9_2", seed)
    say("quorum (9,2) seed", seed, "q", q)
    got = ctx.solve_quorum(inst.seqs, inst.n, inst.m, inst.l, inst.d, q)
    want = oracle.q1(inst.seqs, inst.n, inst.m, inst.l, inst.d, q)
    assert got.shape == want.shape and (got == want).all()


@pytest.mark.parametrize("seed,q", [(1, 10), (1, 15), (2, 5)])
def test_quorum_stored_sets(ctx, seed, q):
    # stored by tests/golden/make_golden.py from the oracle (Q1 = Q0)
    kv = {}
    for line in open(os.path.join(GOLDEN, "pms_9_2_seed%d_q%d.txt" % (seed, q))):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    inst = pmsgen.plain("pms_9_2", seed)
    got = ctx.solve_quorum(inst.seqs, inst.n, inst.m, inst.l, inst.d, q)
    assert len(got) == int(kv["count"])
    assert hashlib.sha256(got.astype("<u8").tobytes()).hexdigest() == \
        kv["codes_sha256"]


def test_quorum_random_small(ctx):
    rng = random.Random(31)
    for case in range(24):
        l = rng.randint(3, 10)
        d = rng.randint(0, min(l - 1, 3))
        n = rng.randint(2, 14)
        m = rng.randint(l, 90)
        q = rng.randint(1, n - 1)
        seqs = bytes(rng.choice(ACGT) for _ in range(n * m))
        say("quorum random case", case, (n, m, l, d, q))
        got = ctx.solve_quorum(seqs, n, m, l, d, q)
        want = oracle.q1(seqs, n, m, l, d, q)
        assert got.shape == want.shape and (got == want).all(), \
            (n, m, l, d, q)


def test_quorum_q_equal_n_is_pms(ctx):
    inst = pmsgen.plain("pms_13_4", 1)
    a = ctx.solve_quorum(inst.seqs, inst.n, inst.m, inst.l, inst.d, inst.n)
    b = ctx.solve(inst.seqs, inst.n, inst.m, inst.l, inst.d)
    assert (a == b).all() and code_of(inst.motif) in set(a.tolist())


def test_quorum_edges(ctx):
    rng = random.Random(3)
    # the largest allowed miss budget: n - q = 30
    n, m, l, d = 31, 40, 6, 1
    seqs = bytes(rng.choice(ACGT) for _ in range(n * m))
    got = ctx.solve_quorum(seqs, n, m, l, d, 1)
    assert (got == oracle.q1(seqs, n, m, l, d, 1)).all()
    # one string less than all, the plant in every string
    inst = pmsgen.plain("pms_9_2", 1)
    got = ctx.solve_quorum(inst.seqs, inst.n, inst.m, 9, 2, inst.n - 1)
    assert (got == oracle.q1(inst.seqs, inst.n, inst.m, 9, 2,
                             inst.n - 1)).all()
    # l = 3 (a single tile of 4^3 codes), d = 0 (exact occurrences)
    seqs = bytes(rng.choice(ACGT) for _ in range(5 * 12))
    for l, d, q in [(3, 0, 2), (3, 2, 1), (4, 0, 3)]:
        got = ctx.solve_quorum(seqs, 5, 12, l, d, q)
        assert (got == oracle.q1(seqs, 5, 12, l, d, q)).all(), (l, d, q)
    # rejected
    for q in (0, inst.n + 1):
        with pytest.raises(pms.PmsError):
            ctx.solve_quorum(inst.seqs, inst.n, inst.m, 9, 2, q)
    seqs = bytes(rng.choice(ACGT) for _ in range(32 * 30))
    with pytest.raises(pms.PmsError):
        ctx.solve_quorum(seqs, 32, 30, 6, 1, 1)          # n - q = 31
    # beyond the tiles (4^15 of them at l = 23): the sample-driven filter
    seqs = bytes(rng.choice(ACGT) for _ in range(4 * 40))
    got = ctx.solve_quorum(seqs, 4, 40, 23, 3, 2)
    assert ctx.stats()["path"] == pms.PATH_FILTER
    assert (got == oracle.q1(seqs, 4, 40, 23, 3, 2)).all()
    for path in (pms.PATH_BITSET, pms.PATH_PAIR):
        with pms.Context(path=path) as c2:
            with pytest.raises(pms.PmsError):
                c2.solve_quorum(inst.seqs, inst.n, inst.m, 9, 2, 10)
    bad = bytearray(inst.seqs)
    bad[5 * inst.m + 17] = ord("N")
    with pytest.raises(pms.PmsError):
        ctx.solve_quorum(bytes(bad), inst.n, inst.m, 9, 2, 10)


@pytest.fixture(scope="module")
def fctx():
    c = pms.Context(path=pms.PATH_FILTER)
    yield c
    c.close()


def test_quorum_filter_path_random_small(fctx):
    # the sample-driven quorum (references from s_1..s_(n-q+1), a miss
    # count per candidate, each motif kept from its first reference)
    rng = random.Random(31)
    for case in range(40):
        l = rng.randint(3, 9)
        d = rng.randint(0, min(3, l - 1))
        n = rng.randint(2, 9)
        m = rng.randint(l, 50)
        q = rng.randint(1, n - 1)
        seqs = bytes(rng.choice(ACGT) for _ in range(n * m))
        got = fctx.solve_quorum(seqs, n, m, l, d, q)
        assert fctx.stats()["path"] == pms.PATH_FILTER
        want = oracle.q1(seqs, n, m, l, d, q)
        assert got.shape == want.shape and (got == want).all(), \
            (case, n, m, l, d, q)


@pytest.mark.parametrize("seed,q", [(1, 19), (1, 15), (2, 10), (3, 17)])
def test_quorum_filter_path_full_9_2(fctx, ctx, seed, q):
    inst = pmsgen.plain("pms_9_2", seed)
    say("quorum filter (9,2) seed", seed, "q", q)
    got = fctx.solve_quorum(inst.seqs, inst.n, inst.m, 9, 2, q)
    want = oracle.q1(inst.seqs, inst.n, inst.m, 9, 2, q)
    assert got.shape == want.shape and (got == want).all()
    assert (ctx.solve_quorum(inst.seqs, inst.n, inst.m, 9, 2, q) == got).all()


def test_quorum_filter_path_long_motifs(ctx):
    # l beyond the tiled path (23..32): the automatic choice is the filter
    for (n, m, l, d, q) in [(5, 40, 24, 2, 3), (6, 45, 28, 3, 4),
                            (4, 50, 32, 2, 2), (7, 40, 25, 1, 5)]:
        inst = pmsgen.planted(l * 3 + d, n, m, l, d)
        say("quorum long", (n, m, l, d, q))
        got = ctx.solve_quorum(inst.seqs, n, m, l, d, q)
        assert ctx.stats()["path"] == pms.PATH_FILTER
        want = oracle.q1(inst.seqs, n, m, l, d, q)
        assert got.shape == want.shape and (got == want).all(), (l, d, q)
        assert code_of(inst.motif) in set(int(v) for v in got)


def test_quorum_filter_equals_tiled_13_4(fctx, ctx):
    # (13,4), n = 20, m = 600, q = 15: the two exact quorum paths agree code
    # for code; sampled codes are checked against the oracle's count
    inst = pmsgen.plain("pms_13_4", 1)
    n, m, l, d, q = inst.n, inst.m, 13, 4, 15
    tiled = ctx.solve_quorum(inst.seqs, n, m, l, d, q)
    filt = fctx.solve_quorum(inst.seqs, n, m, l, d, q)
    assert fctx.stats()["path"] == pms.PATH_FILTER
    say("quorum (13,4,15):", len(tiled), "motifs")
    assert tiled.shape == filt.shape and (tiled == filt).all()
    rng = random.Random(5)
    for c in rng.sample(list(tiled), min(200, len(tiled))):
        assert oracle.hit_count(inst.seqs, n, m, l, d, int(c)) >= q


def test_quorum_largest_l(ctx):
    # l = 22 with tiles of 4^8 codes is 4^14 tiles, the most the quorum path
    # takes (l = 23 is rejected above); strings are near-copies of two random
    # strings (one base redrawn each), so the sets are dense
    rng = random.Random(22)
    pool = [bytes(rng.choice(ACGT) for _ in range(30)) for _ in range(2)]
    for n, q in [(4, 2), (5, 3)]:
        seqs = bytearray()
        for i in range(n):
            s = bytearray(pool[i % 2])
            s[rng.randrange(30)] = rng.choice(ACGT)
            seqs += s
        seqs = bytes(seqs)
        want = oracle.q1(seqs, n, 30, 22, 3, q)
        assert len(want) > 10000
        say("quorum l=22 n", n, "q", q)
        got = ctx.solve_quorum(seqs, n, 30, 22, 3, q)
        assert got.shape == want.shape and (got == want).all(), (n, q)
        st = ctx.stats()
        assert st["tile_suffix"] == 8 and st["tiles"] == 4 ** 14


def test_quorum_order_invariance(ctx):
    inst = pmsgen.plain("pms_9_2", 2)
    rows = [inst.seqs[i * inst.m:(i + 1) * inst.m] for i in range(inst.n)]
    perm = list(range(inst.n))
    random.Random(8).shuffle(perm)
    sh = b"".join(rows[i] for i in perm)
    a = ctx.solve_quorum(inst.seqs, inst.n, inst.m, 9, 2, 11)
    b = ctx.solve_quorum(sh, inst.n, inst.m, 9, 2, 11)
    assert (a == b).all()


def check_large(ctx, name, q, samples):
    """Full-size quorum instance: properties the oracle checks one code at
    a time."""
    import torch
    inst = pmsgen.plain(name, 1)
    n, m, l, d = inst.n, inst.m, inst.l, inst.d
    dev = torch.device("cuda:0")
    d_seqs = torch.frombuffer(bytearray(inst.seqs), dtype=torch.uint8).to(dev)
    cap = 1 << 16
    while True:
        d_out = torch.empty(cap, dtype=torch.int64, device=dev)
        try:
            cnt = ctx.solve_quorum_device(d_seqs.data_ptr(), n, m, l, d, q,
                                          d_out.data_ptr(), cap)
            break
        except pms.PmsError as e:
            assert getattr(e, "needed", 0) > cap
            cap = e.needed
            del d_out
    say(name, "q", q, "motifs", cnt)
    out = d_out[:cnt]
    assert cnt > 0
    assert bool((out[1:] > out[:-1]).all())        # ascending, no repeats
    assert int(out[-1]) < 4 ** l
    host = out.cpu().numpy().astype(np.uint64)

    def member(c):
        j = int(np.searchsorted(host, np.uint64(c)))
        return j < cnt and int(host[j]) == c

    rng = random.Random(17)
    for i in rng.sample(range(cnt), min(samples, cnt)):
        assert oracle.hit_count(inst.seqs, n, m, l, d, int(host[i])) >= q
    nonmember = 0
    while nonmember < samples:
        c = rng.randrange(4 ** l)
        if not member(c):
            assert oracle.hit_count(inst.seqs, n, m, l, d, c) < q
            nonmember += 1
    assert member(code_of(inst.motif))
    return host


def test_quorum_13_4_q10_full_size(ctx):
    a = check_large(ctx, "pms_13_4", 10, 300)
    inst = pmsgen.plain("pms_13_4", 1)
    b = ctx.solve_quorum(inst.seqs, inst.n, inst.m, 13, 4, 12)
    assert np.isin(b, a).all()                       # monotone in q


def test_quorum_17_6_q10_full_size(ctx):
    check_large(ctx, "pms_17_6", 10, 150)
