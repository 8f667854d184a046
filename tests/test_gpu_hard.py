"""GPU: the harder instances of the thesis's Table 3.3, (19,7), (21,8) and
(23,9) with n = 20, m = 600, on the tiled path.

The oracle cannot recompute these sets whole (one reference's sphere at
(21,8) is 1.6e9 candidates), so: at (19,7) the tiled path must equal the
sample-driven filter path (a different algorithm) code for code; at every
size each reported code is checked against every string by the oracle, one
code at a time, and the planted motif must be reported.
"""
import sys

import pytest

import oracle
import paper_2403_00306_amd as pms
import pmsgen

pytestmark = pytest.mark.gpu

ACGT = b"ACGT"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def code_of(lmer: bytes) -> int:
    c = 0
    for ch in lmer:
        c = 4 * c + ACGT.index(ch)
    return c


def check(inst, got):
    assert list(got) == sorted(set(int(v) for v in got))
    for v in got:
        assert oracle.is_motif(inst.seqs, inst.n, inst.m, inst.l, inst.d,
                               int(v))
    assert code_of(inst.motif) in set(int(v) for v in got)


def test_hard_19_7_paths_agree():
    inst = pmsgen.planted(1, 20, 600, 19, 7)
    say("hard (19,7) tiled")
    with pms.Context(path=pms.PATH_TILED) as c:
        tiled = c.solve(inst.seqs, 20, 600, 19, 7)
    say("hard (19,7) filter")
    with pms.Context(path=pms.PATH_FILTER) as c:
        filt = c.solve(inst.seqs, 20, 600, 19, 7)
    assert list(tiled) == list(filt)
    check(inst, tiled)


def test_hard_21_8():
    inst = pmsgen.planted(1, 20, 600, 21, 8)
    say("hard (21,8) tiled")
    with pms.Context(path=pms.PATH_TILED) as c:
        got = c.solve(inst.seqs, 20, 600, 21, 8)
        assert c.stats()["tiles"] == 4 ** 12
    check(inst, got)


def test_hard_23_9():
    inst = pmsgen.planted(1, 20, 600, 23, 9)
    say("hard (23,9) tiled, 4^14 tiles")
    with pms.Context(path=pms.PATH_TILED) as c:
        got = c.solve(inst.seqs, 20, 600, 23, 9)
        assert c.stats()["tiles"] == 4 ** 14
    check(inst, got)
