"""GPU: the harder instances of the thesis's Table 3.3, (19,7), (21,8) and
(23,9) with n = 20, m = 600, on the tiled path.

The oracle cannot recompute these sets in a test (one reference's sphere at
(21,8) is 1.6e9 candidates), so tests/golden/make_golden.py stored them from
the oracle beforehand: the whole (19,7) set (O1 over every reference, with
its canonical Hamming-test count), which the tiled, memory-heavy bitset and
sample-driven filter paths must each equal code for code; and at (19,7) and
(21,8) the motifs derived from single reference l-mers of s_1 (the plant's
offset and two seeded others), each such subset inside the GPU's set, with
the filter path's per-reference canonical counts equal to the oracle's. At
every size each reported code is checked against every string by the
oracle's direct check (Definition 5), one code at a time, and the planted
motif must be reported.
"""
import hashlib
import os
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


def stored_refs(l, d):
    """(offset j, canonical count of j, codes derived from j) per stored
    reference of the (l,d) instance."""
    out = []
    path = os.path.join(os.path.dirname(__file__), "golden",
                        "hard_refs_seed1.txt")
    inst = pmsgen.planted(1, 20, 600, l, d)
    for line in open(path):
        if not line.strip() or line.startswith("#"):
            continue
        t = line.split()
        if (int(t[0]), int(t[1])) != (l, d):
            continue
        assert t[3] == hashlib.sha256(inst.seqs).hexdigest()
        codes = [] if t[6] == "none" else [int(x) for x in t[6].split(",")]
        assert len(codes) == int(t[5])
        out.append((int(t[2]), int(t[4]), codes))
    return out


def check_refs(l, d, got):
    refs = stored_refs(l, d)
    assert len(refs) == 3, "stored references of (%d,%d)" % (l, d)
    have = set(int(v) for v in got)
    for j, _, codes in refs:
        assert set(codes) <= have, (l, d, j)
    return refs


def stored_whole(name, seed):
    """(fields, codes) of a whole motif set stored by make_golden.py."""
    path = os.path.join(os.path.dirname(__file__), "golden",
                        "%s_seed%d.txt" % (name, seed))
    kv = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, v = [t.strip() for t in line.split("=", 1)]
            kv[k] = v
    codes = [int(x) for x in kv["motifs"].split(",") if x]
    assert len(codes) == int(kv["count"])
    return kv, codes


def test_hard_19_7_whole_set():
    inst = pmsgen.planted(1, 20, 600, 19, 7)
    kv, want = stored_whole("pms_19_7", 1)
    assert kv["input_sha256"] == hashlib.sha256(inst.seqs).hexdigest()
    say("hard (19,7) tiled")
    with pms.Context(path=pms.PATH_TILED) as c:
        tiled = c.solve(inst.seqs, 20, 600, 19, 7)
    assert [int(v) for v in tiled] == want
    say("hard (19,7) bitset, 4^19 bits")
    with pms.Context(path=pms.PATH_BITSET) as c:
        bits = c.solve(inst.seqs, 20, 600, 19, 7)
    assert [int(v) for v in bits] == want
    say("hard (19,7) filter")
    with pms.Context(path=pms.PATH_FILTER) as c:
        filt = c.solve(inst.seqs, 20, 600, 19, 7)
        assert c.stats()["hcanon"] == int(kv["hcanon"])
        per = c.hcanon_per_ref(600 - 19 + 1)
    assert [int(v) for v in filt] == want
    check(inst, tiled)
    for j, h, _ in check_refs(19, 7, tiled):
        assert int(per[j]) == h, j


def test_hard_21_8():
    inst = pmsgen.planted(1, 20, 600, 21, 8)
    say("hard (21,8) tiled")
    with pms.Context(path=pms.PATH_TILED) as c:
        got = c.solve(inst.seqs, 20, 600, 21, 8)
        assert c.stats()["tiles"] == 4 ** 12
    check(inst, got)
    check_refs(21, 8, got)


def test_hard_23_9():
    inst = pmsgen.planted(1, 20, 600, 23, 9)
    say("hard (23,9) tiled, 4^14 tiles")
    with pms.Context(path=pms.PATH_TILED) as c:
        got = c.solve(inst.seqs, 20, 600, 23, 9)
        assert c.stats()["tiles"] == 4 ** 14
    check(inst, got)
