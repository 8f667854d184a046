"""The no-allocation entry point (pms_solve_device_noalloc) against
pms_solve_device on the same device buffers: two calls in a row, the second
on a smaller instance (the fixed scratch keeps the first call's contents),
both checked element by element, and against the oracle where it is
cheap."""
import sys

import numpy as np
import pytest

import oracle
import paper_2403_00306_amd as pms
import pmsgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(torch, inst):
    return torch.frombuffer(bytearray(inst.seqs),
                            dtype=torch.uint8).to("cuda:0")


def test_noalloc_matches_solve_device_twice():
    import torch
    big = pmsgen.plain("pms_17_6", 2)              # 4^8 tiles of 4^9 codes
    small = pmsgen.planted(5, 12, 300, 11, 3)      # 4^6 tiles, fewer codes
    cap = 1 << 16
    out_a = torch.zeros(cap, dtype=torch.int64, device="cuda:0")
    out_b = torch.zeros(cap, dtype=torch.int64, device="cuda:0")
    with pms.Context() as c:
        for inst in (big, small):
            say("noalloc", inst.n, inst.m, inst.l, inst.d)
            ds = _dev(torch, inst)
            torch.cuda.synchronize()
            na = c.solve_device_noalloc(ds.data_ptr(), inst.n, inst.m,
                                        inst.l, inst.d, out_a.data_ptr(), cap)
            assert c.stats()["path"] == pms.PATH_TILED
            nb = c.solve_device(ds.data_ptr(), inst.n, inst.m, inst.l, inst.d,
                                out_b.data_ptr(), cap)
            got = out_a[:na].cpu().numpy().view(np.uint64)
            want = out_b[:nb].cpu().numpy().view(np.uint64)
            np.testing.assert_array_equal(got, want)
            if inst.l <= 13:
                np.testing.assert_array_equal(
                    got, oracle.o1(inst.seqs, inst.n, inst.m, inst.l,
                                   inst.d)[0])


def test_noalloc_dense_output_and_limits():
    import torch
    # a dense set (near-copies of one random string): many codes per tile
    # through the scratch heap, then the host-side rejections
    rng = np.random.default_rng(3)
    base = rng.integers(0, 4, 300)
    rows = []
    for i in range(4):
        r = base.copy()
        r[rng.integers(0, 300)] = rng.integers(0, 4)
        rows.append(bytes(b"ACGT"[v] for v in r))
    seqs = b"".join(rows)
    n, m, l, d = 4, 300, 12, 3
    cap = 1 << 22
    out = torch.zeros(cap, dtype=torch.int64, device="cuda:0")
    ds = torch.frombuffer(bytearray(seqs), dtype=torch.uint8).to("cuda:0")
    torch.cuda.synchronize()
    want = oracle.o1(seqs, n, m, l, d)[0]
    assert len(want) > 100000
    with pms.Context() as c:
        cnt = c.solve_device_noalloc(ds.data_ptr(), n, m, l, d,
                                     out.data_ptr(), cap)
        np.testing.assert_array_equal(
            out[:cnt].cpu().numpy().view(np.uint64), want)
        # output capacity too small: PMS_ENOMEM with the size needed
        with pytest.raises(pms.PmsError) as e:
            c.solve_device_noalloc(ds.data_ptr(), n, m, l, d,
                                   out.data_ptr(), 10)
        assert e.value.status == pms.PMS_ENOMEM
        assert getattr(e.value, "needed", 0) == len(want)
        # more tiles than the fixed scratch holds: rejected before launching
        hard = pmsgen.planted(1, 20, 600, 21, 8)
        dh = _dev(torch, hard)
        torch.cuda.synchronize()
        with pytest.raises(pms.PmsError) as e:
            c.solve_device_noalloc(dh.data_ptr(), 20, 600, 21, 8,
                                   out.data_ptr(), cap)
        assert e.value.status == pms.PMS_ENOMEM
        assert "scratch" in str(e.value)
        # outside the tiled path
        with pytest.raises(pms.PmsError) as e:
            c.solve_device_noalloc(ds.data_ptr(), n, m, 2, 1,
                                   out.data_ptr(), cap)
        assert e.value.status == pms.PMS_EINVAL
        # and the ordinary entry point still works after all of that
        cnt2 = c.solve_device(ds.data_ptr(), n, m, l, d, out.data_ptr(), cap)
        np.testing.assert_array_equal(
            out[:cnt2].cpu().numpy().view(np.uint64), want)
