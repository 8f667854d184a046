"""Pins for the pair-based oracle P1 (Observation 3.3, q = n).

P1 must return the motif set of the (separately pinned) sample-driven
oracle O1, and its candidate count must be the sum over the compatible pairs
(x in s_1, y in s_2, d_H(x,y) <= 2d) of the closed-form size of
B(x,d) ∩ B(y,d), with the pairs and their distances computed here.
"""
import math
import random

import numpy as np
import pytest

import oracle
import pmsgen

ACGT = b"ACGT"


def py_dh(a, b):
    return sum(x != y for x, y in zip(a, b))


def pair_intersection(l, d, D):
    """|B(x,d) ∩ B(y,d)| at d_H(x,y) = D, by cases (see the quorum pins,
    where the same count is checked against enumeration)."""
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


def expected_candidates(seqs, m, l, d):
    s1, s2 = seqs[:m], seqs[m:2 * m]
    L = m - l + 1
    tot = 0
    for j in range(L):
        x = s1[j:j + l]
        for k in range(L):
            D = py_dh(x, s2[k:k + l])
            if D <= 2 * d:
                tot += pair_intersection(l, d, D)
    return tot


def test_random_instances_equal_o1():
    rng = random.Random(11)
    for _ in range(30):
        l = rng.randint(3, 8)
        d = rng.randint(0, min(2, l - 1))
        n = rng.randint(2, 7)
        m = rng.randint(l, 40)
        seqs = bytes(rng.choice(ACGT) for _ in range(n * m))
        want, _ = oracle.o1(seqs, n, m, l, d)
        got, nc = oracle.p1(seqs, n, m, l, d)
        assert (got == want).all(), (n, m, l, d)
        assert nc == expected_candidates(seqs, m, l, d)


@pytest.mark.parametrize("rows,l,d", [
    ([b"A" * 20] * 4, 5, 1),                      # one letter
    ([b"ACGT" * 5, b"CGTA" * 5, b"GTAC" * 5], 6, 2),   # periodic
    ([b"ACGTTGCA" * 3, b"TTTTACGT" * 3], 7, 0),   # d = 0: shared l-mers
])
def test_adversarial(rows, l, d):
    seqs = b"".join(rows)
    n, m = len(rows), len(rows[0])
    want, _ = oracle.o1(seqs, n, m, l, d)
    got, nc = oracle.p1(seqs, n, m, l, d)
    assert (got == want).all()
    assert nc == expected_candidates(seqs, m, l, d)


def test_full_size_9_2_and_fewer_candidates():
    inst = pmsgen.plain("pms_9_2", 2)
    got, nc = oracle.p1(inst.seqs, 20, 600, 9, 2)
    want, _ = oracle.o1(inst.seqs, 20, 600, 9, 2)
    assert (got == want).all()
    # fewer candidates than the spheres of all of s_1's l-mers
    assert nc < (600 - 9 + 1) * oracle.nb(9, 2)


def test_needs_two_strings():
    with pytest.raises(oracle.OracleError):
        oracle.p1(b"ACGTACGT", 1, 8, 4, 1)
