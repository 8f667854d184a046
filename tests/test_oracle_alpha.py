"""Pins for the any-alphabet oracle (S1 sample-driven, S0 brute force).

The problem is defined over any alphabet (Sec. 1.2.5) and Table 3.1 gives
the sphere size for any |Sigma|. Expected values come from a literal
pure-Python reading of Definition 5, from the closed-form sphere size, from
the already pinned DNA oracle, and from relabelling invariance.
"""
import itertools
import os
import random

import numpy as np
import pytest

import oracle
import pmsgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def py_dh(a, b):
    return sum(x != y for x, y in zip(a, b))


def py_motifs(rows, alphabet, l, d):
    """Definition 5 (q = n), literally, codes in base |alphabet|."""
    sig = len(alphabet)
    out = []
    for tup in itertools.product(range(sig), repeat=l):
        M = bytes(alphabet[t] for t in tup)
        if all(any(py_dh(M, s[j:j + l]) <= d for j in range(len(s) - l + 1))
               for s in rows):
            c = 0
            for t in tup:
                c = c * sig + t
            out.append(c)
    return out


def test_dna_alphabet_is_the_dna_oracle():
    rng = random.Random(4)
    for _ in range(10):
        l = rng.randint(4, 7)
        d = rng.randint(0, 2)
        n = rng.randint(1, 6)
        m = rng.randint(l, 30)
        seqs = bytes(rng.choice(b"ACGT") for _ in range(n * m))
        o1, _ = oracle.o1(seqs, n, m, l, d)
        assert (oracle.s1(seqs, b"ACGT", n, m, l, d) == o1).all()
        assert (oracle.s0(seqs, b"ACGT", n, m, l, d) == o1).all()


@pytest.mark.parametrize("alphabet", [b"01", b"xyz", b"ABCDE", b"acdefgh"])
def test_tiny_instances_match_definition(alphabet):
    rng = random.Random(len(alphabet))
    for _ in range(12):
        l = rng.randint(1, 4)
        d = rng.randint(0, l - 1)
        n = rng.randint(1, 4)
        m = rng.randint(l, l + 5)
        rows = [bytes(rng.choice(alphabet) for _ in range(m))
                for _ in range(n)]
        seqs = b"".join(rows)
        want = py_motifs(rows, alphabet, l, d)
        assert [int(v) for v in oracle.s1(seqs, alphabet, n, m, l, d)] == want
        assert [int(v) for v in oracle.s0(seqs, alphabet, n, m, l, d)] == want


@pytest.mark.parametrize("l,d", [(3, 1), (4, 2), (5, 3), (6, 2)])
def test_one_lmer_gives_the_sphere(l, d):
    # n = 1, m = l: the motif set is B(x,d), of size sum C(l,k)(sigma-1)^k
    x = bytes(pmsgen.PROTEIN[(7 * j) % 20] for j in range(l))
    got = oracle.s1(x, pmsgen.PROTEIN, 1, l, l, d)
    assert len(got) == oracle.nb(l, d, 20)


def test_protein_sphere_size_by_enumeration():
    # the closed form at sigma = 20 against a literal count (l = 3)
    x = b"KWQ"
    cnt = sum(py_dh(bytes(t), x) <= 2
              for t in itertools.product(pmsgen.PROTEIN, repeat=3))
    assert cnt == oracle.nb(3, 2, 20) == 1 + 3 * 19 + 3 * 19 * 19


def test_relabelling_maps_the_set():
    inst = pmsgen.planted_alpha(3, 6, 30, 5, 1, b"ABCDEFG")
    perm = b"GFEDCBA"            # the same letters in another order
    a = oracle.s1(inst.seqs, b"ABCDEFG", 6, 30, 5, 1)
    b = oracle.s1(inst.seqs, perm, 6, 30, 5, 1)

    def digits(c, sig=7, l=5):
        return [(int(c) // sig ** (l - 1 - j)) % sig for j in range(l)]

    # letter i of the first alphabet is letter 6-i of the second
    mapped = sorted(int(sum((6 - t) * 7 ** (4 - j)
                            for j, t in enumerate(digits(c))))
                    for c in a)
    assert mapped == [int(v) for v in b]
    assert len(a) > 0


def test_plant_found_and_outputs_valid():
    inst = pmsgen.planted_alpha(2, 8, 60, 6, 2)
    got = oracle.s1(inst.seqs, pmsgen.PROTEIN, 8, 60, 6, 2)
    pc = 0
    for ch in inst.motif:
        pc = pc * 20 + pmsgen.PROTEIN.index(ch)
    assert pc in set(int(v) for v in got)


def test_rejects():
    seqs = b"ACDE" * 5
    with pytest.raises(oracle.OracleError):
        oracle.s1(seqs, b"ACDA", 1, 20, 4, 1)          # repeated letter
    with pytest.raises(oracle.OracleError):
        oracle.s1(seqs, b"ACD", 1, 20, 4, 1)           # E not a letter
    with pytest.raises(oracle.OracleError):
        oracle.s1(b"A" * 20, pmsgen.PROTEIN, 1, 20, 15, 1)   # 20^15 > 2^64


def read_kv(path):
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    return kv


def test_golden_protein():
    kv = read_kv(os.path.join(GOLDEN, "protein_8_3_seed1.txt"))
    inst = pmsgen.planted_alpha(1, 20, 600, 8, 3)
    import hashlib
    assert hashlib.sha256(inst.seqs).hexdigest() == kv["input_sha256"]
    # the stored set (written by S1, too slow to rerun here) holds the plant
    assert int(kv["planted_code"]) in [int(x) for x in
                                       kv["motifs"].split(",")]
