"""GPU parity: the HIP library against the CPU oracle, bit for bit.

Every case compares the ascending uint64 motif codes element by element with
the oracle on the same seeded input. Small cases span many tiles and a
ragged tail; the full (9,2) and (13,4) configurations are compared whole;
(17,6) is compared whole with stored oracle sets (seeds 1-5) and also
checked on properties the oracle can verify at any size (every reported
code, the plant, path agreement, and completeness on a sample of reference
l-mers). Integer results: the tolerance is zero.
"""
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
PATHS = [pms.PATH_FILTER, pms.PATH_TILED, pms.PATH_BITSET]


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


def oracle_set(seqs, n, m, l, d):
    return oracle.o1(seqs, n, m, l, d)[0]


def solve_path(path, seqs, n, m, l, d):
    with pms.Context(path=path) as c:
        got = c.solve(seqs, n, m, l, d)
        st = c.stats()
    return got, st


def rand_instance(rng, n, m, alphabet=ACGT):
    return bytes(rng.choice(alphabet) for _ in range(n * m))


# ---------------------------------------------------------------------------
# small and ragged cases, every path
# ---------------------------------------------------------------------------

SMALL = [
    # (n, m, l, d, note)
    (5, 40, 5, 1, "tiny"),
    (8, 61, 7, 2, "ragged m"),
    (6, 33, 6, 0, "d=0"),
    (1, 30, 6, 2, "n=1: union of spheres"),
    (4, 8, 8, 3, "m=l"),
    (7, 95, 9, 2, "several tiles"),
    (3, 1500, 8, 2, "m above one staging chunk"),
    (10, 130, 11, 3, "many tiles"),
    (5, 64, 3, 1, "l=3: one word"),
    (4, 40, 4, 3, "d=l-1"),
    (6, 200, 10, 1, "small d"),
]


@pytest.mark.parametrize("n,m,l,d,note", SMALL)
@pytest.mark.parametrize("path", PATHS)
def test_small_vs_oracle(path, n, m, l, d, note):
    rng = random.Random(hash((n, m, l, d)) & 0xffff)
    seqs = rand_instance(rng, n, m)
    say("case", note, n, m, l, d, "path", path)
    want = oracle_set(seqs, n, m, l, d)
    got, st = solve_path(path, seqs, n, m, l, d)
    assert st["path"] == path
    assert got.dtype == np.uint64
    np.testing.assert_array_equal(got, want)


def test_small_vs_bruteforce_o0():
    rng = random.Random(17)
    for trial in range(12):
        l = rng.randint(3, 8)
        d = rng.randint(0, min(3, l - 1))
        n = rng.randint(1, 6)
        m = rng.randint(l, 70)
        seqs = rand_instance(rng, n, m)
        want = oracle.o0(seqs, n, m, l, d)
        for path in PATHS:
            got, _ = solve_path(path, seqs, n, m, l, d)
            np.testing.assert_array_equal(got, want, err_msg=str(
                (trial, path, n, m, l, d)))


def test_long_motifs_filter_path():
    # l up to 32 (one 32-bit word per bit plane); the planner picks the
    # sample-driven path here
    for (n, m, l, d) in [(4, 60, 32, 2), (5, 80, 20, 3), (3, 50, 25, 1)]:
        inst = pmsgen.planted(l * 7 + d, n, m, l, d)
        want = oracle_set(inst.seqs, n, m, l, d)
        with pms.Context() as c:
            got = c.solve(inst.seqs, n, m, l, d)
        np.testing.assert_array_equal(got, want)
        assert code_of(inst.motif) in set(int(x) for x in got)


def test_low_entropy_inputs_many_motifs():
    # two-letter strings: large outputs exercise the radix sort and the
    # output-capacity retry
    rng = random.Random(5)
    n, m, l, d = 3, 300, 9, 3
    seqs = rand_instance(rng, n, m, alphabet=b"AC")
    want = oracle_set(seqs, n, m, l, d)
    assert len(want) > 4096
    for path in PATHS:
        got, st = solve_path(path, seqs, n, m, l, d)
        np.testing.assert_array_equal(got, want)


def test_n1_huge_output_tiled_and_filter():
    rng = random.Random(8)
    n, m, l, d = 1, 400, 10, 3
    seqs = rand_instance(rng, n, m)
    want = oracle_set(seqs, n, m, l, d)
    assert len(want) > 100000
    for path in (pms.PATH_TILED, pms.PATH_FILTER):
        got, _ = solve_path(path, seqs, n, m, l, d)
        np.testing.assert_array_equal(got, want)


# ---------------------------------------------------------------------------
# the thesis-sized configurations (Table 3.2: n = 20, m = 600)
# ---------------------------------------------------------------------------

def load_golden(name, seed):
    path = os.path.join(os.path.dirname(__file__), "golden",
                        "%s_seed%d.txt" % (name, seed))
    kv = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, v = [t.strip() for t in line.split("=", 1)]
            kv[k] = v
    return kv, np.array([int(x) for x in kv["motifs"].split(",") if x],
                        dtype=np.uint64)


# every seed of the three plain configurations, stored by
# tests/golden/make_golden.py from the oracle (O1, and O0 where l <= 13)
GOLDEN_PLAIN = ([("pms_9_2", k) for k in range(1, 6)] +
                [("pms_13_4", k) for k in range(1, 6)] +
                [("pms_17_6", k) for k in range(1, 6)])


@pytest.mark.parametrize("name,seed", GOLDEN_PLAIN)
@pytest.mark.parametrize("path", PATHS)
def test_full_size_golden(name, seed, path):
    kv, want = load_golden(name, seed)
    inst = pmsgen.plain(name, seed)
    import hashlib
    assert hashlib.sha256(inst.seqs).hexdigest() == kv["input_sha256"]
    say("full", name, seed, "path", path)
    got, st = solve_path(path, inst.seqs, inst.n, inst.m, inst.l, inst.d)
    np.testing.assert_array_equal(got, want)
    assert code_of(inst.motif) in set(int(x) for x in got)
    if path == pms.PATH_FILTER:
        assert st["hcanon"] == int(kv["hcanon"])


@pytest.mark.parametrize("seed", [2, 3])
def test_13_4_more_seeds(seed):
    inst = pmsgen.plain("pms_13_4", seed)
    want, h = oracle.o1(inst.seqs, inst.n, inst.m, inst.l, inst.d)
    for path in (pms.PATH_TILED, pms.PATH_FILTER):
        got, st = solve_path(path, inst.seqs, inst.n, inst.m, inst.l, inst.d)
        np.testing.assert_array_equal(got, want)
        if path == pms.PATH_FILTER:
            assert st["hcanon"] == h
            # executed tests: whole waves (multiples of 64), same order of
            # magnitude as the canonical count
            ex = st["filter_tests"]
            assert ex > 0 and ex % 64 == 0
            assert 0.2 * h <= ex <= 20 * h, (ex, h)


def test_17_6_properties():
    inst = pmsgen.plain("pms_17_6", 1)
    n, m, l, d = inst.n, inst.m, inst.l, inst.d
    say("full 17,6 tiled")
    tiled, _ = solve_path(pms.PATH_TILED, inst.seqs, n, m, l, d)
    say("full 17,6 bitset")
    bitset, _ = solve_path(pms.PATH_BITSET, inst.seqs, n, m, l, d)
    np.testing.assert_array_equal(tiled, bitset)
    assert np.all(np.diff(tiled.astype(np.int64)) > 0)
    # every reported code is a motif (direct check, Definitions 4-5)
    for c in tiled:
        assert oracle.is_motif(inst.seqs, n, m, l, d, int(c))
    assert code_of(inst.motif) in set(int(x) for x in tiled)
    # completeness on sampled references: what the oracle derives from these
    # l-mers of s_1 must all be reported; the filter path's per-reference
    # Hamming-test counts match the oracle's on the same references
    say("full 17,6 filter")
    with pms.Context(path=pms.PATH_FILTER) as c:
        filt = c.solve(inst.seqs, n, m, l, d)
        per = c.hcanon_per_ref(m - l + 1)
    np.testing.assert_array_equal(filt, tiled)
    rng = random.Random(3)
    refs = sorted(rng.sample(range(m - l + 1), 3)) + [inst.positions[0]]
    for j in refs:
        part, h, pr = oracle.o1(inst.seqs, n, m, l, d, ref_begin=j,
                                ref_end=j + 1, per_ref=True)
        assert set(int(x) for x in part) <= set(int(x) for x in tiled)
        assert int(per[j]) == h


# ---------------------------------------------------------------------------
# tile shape invariance, determinism, device entry point, errors
# ---------------------------------------------------------------------------

def test_tile_shapes_do_not_change_result():
    inst = pmsgen.planted(4, 12, 300, 11, 3)
    want = oracle_set(inst.seqs, inst.n, inst.m, 11, 3)
    with pms.Context(path=pms.PATH_TILED) as c:
        for s in range(3, 10):
            for t in (1, 32, 256):
                c.set_tile_config(11, 3, s, t)
                got = c.solve(inst.seqs, inst.n, inst.m, 11, 3)
                np.testing.assert_array_equal(got, want, err_msg="s=%d t=%d"
                                              % (s, t))
                assert c.stats()["tile_suffix"] == s


@pytest.mark.parametrize("threads", [256, 512])
def test_tile_kernel_sizes_vs_oracle(threads):
    # both workgroup sizes of the tile kernel, forced, on every tile suffix
    # (the automatic choice takes 512 threads only for s = 9)
    inst = pmsgen.planted(5, 12, 300, 11, 3)
    want = oracle_set(inst.seqs, inst.n, inst.m, 11, 3)
    with pms.Context(path=pms.PATH_TILED, tile_threads=threads) as c:
        for s in (3, 6, 8, 9):
            for t in (1, 64, 256):
                c.set_tile_config(11, 3, s, t)
                got = c.solve(inst.seqs, inst.n, inst.m, 11, 3)
                np.testing.assert_array_equal(
                    got, want, err_msg="threads=%d s=%d t=%d" % (threads, s, t))
                assert c.stats()["tile_threads"] == threads


def test_tile_kernel_sizes_agree_17_6():
    inst = pmsgen.plain("pms_17_6", 1)
    res = {}
    for threads in (0, 256, 512):
        with pms.Context(path=pms.PATH_TILED, tile_threads=threads) as c:
            res[threads] = c.solve(inst.seqs, 20, 600, 17, 6)
            st = c.stats()
        say("(17,6) threads", threads, "->", st["tile_threads"], "ms",
            st["ms_main"])
        assert st["tile_threads"] == (threads or 512)
    np.testing.assert_array_equal(res[256], res[512])
    np.testing.assert_array_equal(res[0], res[512])
    with pytest.raises(pms.PmsError):
        pms.Context(tile_threads=128)


def test_tile_order_and_long_strings():
    # s = 9 turns the per-tile string order on (a pass's word marks well
    # above the n*L prefix tests) and L = 990 takes the survivor stage over
    # two register rounds per string; t = 1 and 256 bound its list size
    inst = pmsgen.planted(9, 16, 1000, 11, 3)
    want = oracle_set(inst.seqs, inst.n, inst.m, 11, 3)
    with pms.Context(path=pms.PATH_TILED) as c:
        for t in (1, 64, 256):
            c.set_tile_config(11, 3, 9, t)
            say("order/long t", t)
            got = c.solve(inst.seqs, inst.n, inst.m, 11, 3)
            np.testing.assert_array_equal(got, want, err_msg="t=%d" % t)


def mutated_copies(seed, n, m, k, muts):
    # n strings, each a copy of one of k random strings with `muts` random
    # positions redrawn: dense motif sets in which every string differs
    rng = random.Random(seed)
    pool = [bytearray(rng.choice(ACGT) for _ in range(m)) for _ in range(k)]
    out = bytearray()
    for i in range(n):
        s = bytearray(pool[i % k])
        for _ in range(muts):
            s[rng.randrange(m)] = rng.choice(ACGT)
        out += s
    return bytes(out)


@pytest.mark.parametrize("threads", [256, 512])
def test_string_order_limit_vs_oracle(threads):
    # (16,6) at s = 9: 4^7 tiles, enough for items of four sibling tiles that
    # share one string order (with 4 workgroups per CU); n = 64 is the
    # largest n the per-tile order covers, n = 65 runs in input order
    n_l, n_d, m = 16, 6, 30
    for n in (64, 65):
        seqs = mutated_copies(64 + n, n, m, 2, 1)
        want = oracle_set(seqs, n, m, n_l, n_d)
        assert len(want) > 10000
        with pms.Context(path=pms.PATH_TILED, tile_threads=threads) as c:
            c.set_tile_config(n_l, n_d, 9, 64)
            say("order limit n", n, "threads", threads)
            got = c.solve(seqs, n, m, n_l, n_d)
            assert c.stats()["tile_threads"] == threads
        np.testing.assert_array_equal(got, want, err_msg="n=%d" % n)


def test_bitset_order_limit_vs_oracle():
    # the memory-heavy path orders the strings per tile for n <= 64 and
    # takes them in input order above; (16,6) at s = 9, 4^7 tiles of 4^9 bits
    n_l, n_d, m = 16, 6, 30
    for n in (64, 65):
        seqs = mutated_copies(64 + n, n, m, 2, 1)
        want = oracle_set(seqs, n, m, n_l, n_d)
        say("bitset order limit n", n)
        got, st = solve_path(pms.PATH_BITSET, seqs, n, m, n_l, n_d)
        assert st["tile_suffix"] == 9
        np.testing.assert_array_equal(got, want, err_msg="n=%d" % n)


def test_many_strings_every_path():
    # hundreds of strings (n has no upper limit): near-copies of one random
    # string, one base redrawn in each; every exact path, and the quorum at
    # its largest miss budget n - q = 30
    for (n, m, l, d) in [(300, 25, 9, 2), (1000, 20, 8, 2)]:
        seqs = mutated_copies(n, n, m, 1, 1)
        want = oracle_set(seqs, n, m, l, d)
        assert len(want) > 100
        for path in PATHS + [pms.PATH_PAIR]:
            say("many strings n", n, "path", path)
            got, _ = solve_path(path, seqs, n, m, l, d)
            np.testing.assert_array_equal(got, want,
                                          err_msg="n=%d path=%d" % (n, path))
        wq = oracle.q1(seqs, n, m, l, d, n - 30)
        with pms.Context() as c:
            gq = c.solve_quorum(seqs, n, m, l, d, n - 30)
        np.testing.assert_array_equal(gq, wq, err_msg="quorum n=%d" % n)


def test_tile_count_limit():
    # l = 23 at s = 9 is exactly 4^14 tiles, the most the tiled path takes;
    # at l = 24 a forced tiled solve runs on the filter path instead
    for l in (23, 24):
        seqs = mutated_copies(100 + l, 3, 30, 1, 1)
        want = oracle_set(seqs, 3, 30, l, 3)
        assert len(want) > 10000
        say("tile limit l", l)
        got, st = solve_path(pms.PATH_TILED, seqs, 3, 30, l, 3)
        np.testing.assert_array_equal(got, want, err_msg="l=%d" % l)
        if l == 23:
            assert st["path"] == pms.PATH_TILED
            assert st["tile_suffix"] == 9 and st["tiles"] == 4 ** 14
        else:
            assert st["path"] == pms.PATH_FILTER


def test_repeat_runs_identical(ctx):
    inst = pmsgen.plain("pms_13_4", 4)
    a = ctx.solve(inst.seqs, inst.n, inst.m, inst.l, inst.d)
    for _ in range(3):
        np.testing.assert_array_equal(
            ctx.solve(inst.seqs, inst.n, inst.m, inst.l, inst.d), a)


def test_solve_device_with_torch_buffers(ctx):
    import torch
    inst = pmsgen.plain("pms_13_4", 1)
    _, want = load_golden("pms_13_4", 1)
    dev = torch.device("cuda:0")
    d_seqs = torch.frombuffer(bytearray(inst.seqs), dtype=torch.uint8).to(dev)
    d_out = torch.zeros(1024, dtype=torch.int64, device=dev)
    s = torch.cuda.Stream()
    cnt = ctx.solve_device(d_seqs.data_ptr(), inst.n, inst.m, inst.l, inst.d,
                           d_out.data_ptr(), 1024, stream=s.cuda_stream)
    got = d_out[:cnt].cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, want)
    # capacity too small: PMS_ENOMEM with the size needed
    small = torch.zeros(2, dtype=torch.int64, device=dev)
    with pytest.raises(pms.PmsError) as e:
        ctx.solve_device(d_seqs.data_ptr(), inst.n, inst.m, inst.l, inst.d,
                         small.data_ptr(), 2)
    assert e.value.status == pms.PMS_ENOMEM and e.value.needed == len(want)
    # capacity exactly the size of the set
    exact = torch.zeros(len(want), dtype=torch.int64, device=dev)
    cnt = ctx.solve_device(d_seqs.data_ptr(), inst.n, inst.m, inst.l, inst.d,
                           exact.data_ptr(), len(want))
    assert cnt == len(want)
    np.testing.assert_array_equal(exact.cpu().numpy().view(np.uint64), want)
    # an instance without motifs: count 0, with capacity 0
    rng = random.Random(1)
    none = bytes(rng.choice(ACGT) for _ in range(5 * 20))
    assert len(oracle_set(none, 5, 20, 8, 1)) == 0
    d_none = torch.frombuffer(bytearray(none), dtype=torch.uint8).to(dev)
    assert ctx.solve_device(d_none.data_ptr(), 5, 20, 8, 1,
                            exact.data_ptr(), 0) == 0


def test_error_paths(ctx):
    good = pmsgen.planted(1, 4, 30, 6, 1).seqs
    bad = bytearray(good)
    bad[2 * 30 + 7] = ord("N")
    with pytest.raises(pms.PmsError) as e:
        ctx.solve(bytes(bad), 4, 30, 6, 1)
    assert e.value.status == pms.PMS_EBASE
    assert "string 2 at offset 7" in str(e.value)
    for (n, m, l, d) in [(4, 30, 6, 6), (4, 30, 33, 1), (0, 30, 6, 1),
                         (4, 5, 6, 1), (4, 30, 6, -1)]:
        with pytest.raises(pms.PmsError) as e:
            ctx.solve(b"A" * (n * m), n, m, l, d)
        assert e.value.status == pms.PMS_EINVAL
    # the context still works after errors
    assert len(ctx.solve(good, 4, 30, 6, 1)) >= 1
    # a budget too small for the buffers is reported, not crashed on
    with pms.Context(mem_budget_bytes=1 << 20) as small:
        inst = pmsgen.plain("pms_13_4", 1)
        with pytest.raises(pms.PmsError) as e:
            small.solve(inst.seqs, inst.n, inst.m, inst.l, inst.d)
        assert e.value.status == pms.PMS_ENOMEM
