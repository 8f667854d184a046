"""GPU parity for motifs over other alphabets (pms_solve_alphabet).

The HIP library against the any-alphabet CPU oracle (S1), code for code on
the same seeded inputs: random small instances over 2..32 letters (ragged
sizes, many reference chunks), inputs with many repeats (every motif reached
from many l-mers), DNA in another letter order, the stored full-size protein
set at (8,3), the device-buffer variant and the error cases. Integer
results: the tolerance is zero.
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

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LETTERS = bytes(range(ord("A"), ord("A") + 26)) + b"012345"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = pms.Context()
    yield c
    c.close()


@pytest.mark.parametrize("sigma", [2, 3, 5, 7, 20, 32])
def test_alpha_random_small(ctx, sigma):
    rng = random.Random(100 + sigma)
    alphabet = bytes(rng.sample(list(LETTERS), sigma))
    for case in range(6):
        l = rng.randint(2, 6)
        d = rng.randint(0, min(l - 1, 2))
        n = rng.randint(1, 6)
        m = rng.randint(l, 50)
        seqs = bytes(rng.choice(alphabet) for _ in range(n * m))
        say("alphabet", sigma, "case", case, (n, m, l, d))
        got = ctx.solve_alphabet(alphabet, seqs, n, m, l, d)
        want = oracle.s1(seqs, alphabet, n, m, l, d)
        assert got.shape == want.shape and (got == want).all(), \
            (sigma, n, m, l, d)


def test_alpha_top_of_code_range(ctx):
    # the largest l whose codes fit in 64 bits for each alphabet size: at
    # 4^32 = 16^16 = 2^64 and 9^20 > 2^63 many motif codes have the top bit
    # set (the device sort must order them as unsigned); 20^14 is the protein
    # limit. l + 1 is rejected. Dense sets from near-copies of one string.
    rng = random.Random(71)
    for alphabet, l, m in [(b"ACGT", 32, 40), (LETTERS[:16], 16, 30),
                           (LETTERS[:9], 20, 30), (pmsgen.PROTEIN, 14, 30)]:
        base = bytearray(rng.choice(alphabet) for _ in range(m))
        seqs = bytearray()
        for _ in range(3):
            s = bytearray(base)
            s[rng.randrange(m)] = rng.choice(alphabet)
            seqs += s
        seqs = bytes(seqs)
        say("code range", len(alphabet), l)
        want = oracle.s1(seqs, alphabet, 3, m, l, 2)
        got = ctx.solve_alphabet(alphabet, seqs, 3, m, l, 2)
        assert got.shape == want.shape and (got == want).all(), \
            (len(alphabet), l)
        if len(alphabet) != 20:
            assert (want >= np.uint64(1 << 63)).any()
        with pytest.raises(pms.PmsError):
            ctx.solve_alphabet(alphabet, seqs, 3, m, l + 1, 2)


def test_alpha_repeats(ctx):
    # low-complexity strings: each motif lies in the spheres of many l-mers
    alphabet = pmsgen.PROTEIN
    rows = [b"ACDACDACDACDACDACD" * 2, b"CDACDACDACDACDACDA" * 2,
            b"DACDACDACDACDACDAC" * 2]
    seqs = b"".join(rows)
    for l, d in [(5, 1), (6, 2)]:
        got = ctx.solve_alphabet(alphabet, seqs, 3, 36, l, d)
        want = oracle.s1(seqs, alphabet, 3, 36, l, d)
        assert len(want) > 0 and (got == want).all()


def test_alpha_dna_letter_order(ctx):
    inst = pmsgen.plain("pms_9_2", 1)
    # "ACGT" is pms_solve; another order runs the any-alphabet kernel
    assert (ctx.solve_alphabet(b"ACGT", inst.seqs, 20, 600, 9, 2)
            == ctx.solve(inst.seqs, 20, 600, 9, 2)).all()
    got = ctx.solve_alphabet(b"TGCA", inst.seqs[:8 * 120], 8, 120, 7, 1)
    want = oracle.s1(inst.seqs[:8 * 120], b"TGCA", 8, 120, 7, 1)
    assert (got == want).all()


def test_alpha_canonical_test_count(ctx):
    # relabelling letters maps spheres to spheres and strings to strings, so
    # DNA in another letter order has the DNA oracle's H_canon exactly
    inst = pmsgen.plain("pms_9_2", 2)
    seqs = inst.seqs[:10 * 200]
    ctx.solve_alphabet(b"GATC", seqs, 10, 200, 8, 2)
    _, h = oracle.o1(seqs, 10, 200, 8, 2)
    assert ctx.stats()["hcanon"] == h


def test_alpha_protein_full_size_stored(ctx):
    kv = {}
    for line in open(os.path.join(GOLDEN, "protein_8_3_seed1.txt")):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    inst = pmsgen.planted_alpha(1, 20, 600, 8, 3)
    got = ctx.solve_alphabet(pmsgen.PROTEIN, inst.seqs, 20, 600, 8, 3)
    assert [int(v) for v in got] == [int(x) for x in kv["motifs"].split(",")]


def test_alpha_device_buffers(ctx):
    import torch
    inst = pmsgen.planted_alpha(5, 10, 200, 7, 2)
    dev = torch.device("cuda:0")
    d_seqs = torch.frombuffer(bytearray(inst.seqs), dtype=torch.uint8).to(dev)
    host = ctx.solve_alphabet(pmsgen.PROTEIN, inst.seqs, 10, 200, 7, 2)
    small = torch.zeros(max(len(host) - 1, 1), dtype=torch.int64, device=dev)
    if len(host) > 1:
        with pytest.raises(pms.PmsError) as ei:
            ctx.solve_alphabet_device(pmsgen.PROTEIN, d_seqs.data_ptr(), 10,
                                      200, 7, 2, small.data_ptr(),
                                      small.numel())
        assert ei.value.needed == len(host)
    out = torch.zeros(len(host) + 8, dtype=torch.int64, device=dev)
    cnt = ctx.solve_alphabet_device(pmsgen.PROTEIN, d_seqs.data_ptr(), 10,
                                    200, 7, 2, out.data_ptr(), out.numel())
    assert cnt == len(host)
    assert (out[:cnt].cpu().numpy().view(np.uint64) == host).all()


def test_alpha_errors(ctx):
    inst = pmsgen.planted_alpha(5, 4, 50, 6, 1)
    bad = bytearray(inst.seqs)
    bad[77] = ord("B")                       # not an amino-acid letter
    with pytest.raises(pms.PmsError):
        ctx.solve_alphabet(pmsgen.PROTEIN, bytes(bad), 4, 50, 6, 1)
    with pytest.raises(pms.PmsError):
        ctx.solve_alphabet(b"ACDA", inst.seqs, 4, 50, 6, 1)   # repeated
    with pytest.raises(pms.PmsError):
        ctx.solve_alphabet(LETTERS + b"6", inst.seqs, 4, 50, 6, 1)  # 33
    with pytest.raises(pms.PmsError):
        ctx.solve_alphabet(pmsgen.PROTEIN, b"A" * 4 * 50, 4, 50, 15, 1)
    # the context still works afterwards
    assert len(ctx.solve_alphabet(pmsgen.PROTEIN, inst.seqs, 4, 50, 6, 1)) > 0
