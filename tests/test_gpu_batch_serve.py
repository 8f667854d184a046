"""Batched and served forms: every instance's result equals the oracle's and
the same instance solved alone, bit for bit."""
import random
import sys
import time

import numpy as np
import pytest

import oracle
import paper_2403_00306_amd as pms
import pmsgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed_instances(seed, k, classes, nrange, mrange):
    r = pmsgen.Rng(seed)
    out = []
    for _ in range(k):
        l, d = classes[r.bounded(len(classes))]
        n = nrange[0] + r.bounded(nrange[1] - nrange[0] + 1)
        m = mrange[0] + r.bounded(mrange[1] - mrange[0] + 1)
        out.append(pmsgen.planted(r.next(), n, m, l, d))
    return out


def test_batch_matches_oracle_and_alone():
    insts = mixed_instances(21, 24, [(7, 1), (9, 2), (11, 3), (8, 2)],
                            (3, 12), (40, 300))
    say("batch of", len(insts))
    with pms.Context() as c:
        got = c.solve_batch(insts)
        again = c.solve_batch(insts)      # same shape: graph replay
        alone = [c.solve(x.seqs, x.n, x.m, x.l, x.d) for x in insts]
    for i, x in enumerate(insts):
        want = oracle.o1(x.seqs, x.n, x.m, x.l, x.d)[0]
        np.testing.assert_array_equal(got[i], want, err_msg="inst %d" % i)
        np.testing.assert_array_equal(again[i], want)
        np.testing.assert_array_equal(alone[i], want)


def test_batch_with_quorum_instances():
    # quorum instances (1 <= q < n) in a batch run one by one on their own
    # kernels; plain ones (q = 0 or q = n) in the batched launch; q outside
    # 0..n is a bad instance that does not spoil the others
    plain = mixed_instances(31, 6, [(9, 2), (8, 2)], (4, 10), (60, 200))
    qx = [pmsgen.planted(40 + k, 10, 120, 9, 2) for k in range(3)]
    items = [(x.seqs, x.n, x.m, x.l, x.d) for x in plain]
    items[1] = items[1] + (plain[1].n,)          # q = n: plain search
    items += [(x.seqs, x.n, x.m, x.l, x.d, q)
              for x, q in zip(qx, (3, 7, 9))]
    items.append((qx[0].seqs, 10, 120, 9, 2, 11))   # q > n
    items.append((qx[0].seqs, 10, 120, 9, 2, -1))   # q < 0
    say("batch with quorum instances")
    with pms.Context() as c:
        got = c.solve_batch(items)
    for i, x in enumerate(plain):
        want = oracle.o1(x.seqs, x.n, x.m, x.l, x.d)[0]
        np.testing.assert_array_equal(got[i], want, err_msg="plain %d" % i)
    for k, (x, q) in enumerate(zip(qx, (3, 7, 9))):
        want = oracle.q1(x.seqs, x.n, x.m, x.l, x.d, q)
        np.testing.assert_array_equal(got[len(plain) + k], want,
                                      err_msg="quorum q=%d" % q)
    for bad in got[-2:]:
        assert isinstance(bad, pms.PmsError)
        assert bad.status == pms.PMS_EINVAL


def test_served_rejects_quorum_requests():
    x = pmsgen.planted(5, 6, 80, 9, 2)
    with pms.Context() as c:
        inst = pms.CInstance(x.seqs, 6, 80, 9, 2, 3)
        t = pms.ctypes.c_uint64(0)
        rc = c._lib.pms_submit(c._h, pms.ctypes.byref(inst),
                               pms.ctypes.byref(t))
        assert rc == pms.PMS_EINVAL
        inst.q = 6                                   # q = n: plain request
        assert c._lib.pms_submit(c._h, pms.ctypes.byref(inst),
                                 pms.ctypes.byref(t)) == pms.PMS_OK
        np.testing.assert_array_equal(c.wait(int(t.value), 60000),
                                      oracle.o1(x.seqs, 6, 80, 9, 2)[0])


def test_batch_graph_replays_with_eager_work_between():
    # the first call captures the batch's graph, the next three replay it;
    # a plain solve (other kernels, a host synchronisation) runs between
    # replays, and every replay is checked against the oracle
    insts = mixed_instances(57, 16, [(9, 2), (11, 3), (13, 4)], (4, 10),
                            (50, 200))
    want = [oracle.o1(x.seqs, x.n, x.m, x.l, x.d)[0] for x in insts]
    with pms.Context() as c:
        for rep in range(4):
            got = c.solve_batch(insts)
            assert c.stats()["graph_replayed"] == (1 if rep else 0), rep
            for i in range(len(insts)):
                np.testing.assert_array_equal(
                    got[i], want[i], err_msg="replay %d inst %d" % (rep, i))
            x = insts[rep]
            np.testing.assert_array_equal(
                c.solve(x.seqs, x.n, x.m, x.l, x.d), want[rep])
            assert c.stats()["graph_replayed"] == 0


def test_batch_graph_replay_with_new_contents():
    # the replay key is the batch shape, not the bytes: a second draw of
    # the same (n, m, l, d) shapes must replay the graph and still give the
    # second draw's sets (the input copy and the index are inside the graph)
    shapes = [(x.n, x.m, x.l, x.d) for x in
              mixed_instances(61, 12, [(9, 2), (11, 3), (13, 4)], (4, 12),
                              (60, 250))]
    first = [pmsgen.planted(100 + i, *sh) for i, sh in enumerate(shapes)]
    second = [pmsgen.planted(900 + i, *sh) for i, sh in enumerate(shapes)]
    with pms.Context() as c:
        c.solve_batch(first)
        assert c.stats()["graph_replayed"] == 0
        for rep, insts in enumerate((second, first, second)):
            got = c.solve_batch(insts)
            assert c.stats()["graph_replayed"] == 1, rep
            for i, x in enumerate(insts):
                np.testing.assert_array_equal(
                    got[i], oracle.o1(x.seqs, x.n, x.m, x.l, x.d)[0],
                    err_msg="replay %d inst %d" % (rep, i))


def test_plain_solve_counts_each_retry_once():
    # two-letter strings at (10,3): about 1.1e5 motifs, above the first
    # output estimate (2^16 codes); the first solve retries once, a repeat
    # of the shape starts with the room it needed
    rng = random.Random(2)
    n, m, l, d = 3, 200, 10, 3
    s = bytes(rng.choice(b"AT") for _ in range(n * m))
    want = oracle.o1(s, n, m, l, d)[0]
    with pms.Context(path=pms.PATH_TILED) as c:
        assert len(want) > 1 << 16
        np.testing.assert_array_equal(c.solve(s, n, m, l, d), want)
        assert c.stats()["retries"] == 1
        np.testing.assert_array_equal(c.solve(s, n, m, l, d), want)
        assert c.stats()["retries"] == 0


@pytest.mark.parametrize("threads", [0, 256, 512])
def test_batch_tile_kernel_sizes(threads):
    # (13,4) and (14,4) take tiles of 4^8 and 4^9 codes, where the automatic
    # choice is the 512-thread kernel; forced sizes run every tile with it
    insts = mixed_instances(33, 10, [(9, 2), (13, 4), (14, 4)], (4, 8),
                            (60, 120))
    say("batch threads", threads)
    with pms.Context(tile_threads=threads) as c:
        got = c.solve_batch(insts)
        st = c.stats()
        alone = [c.solve(x.seqs, x.n, x.m, x.l, x.d) for x in insts]
    if st["tiles"] > 0:
        assert st["tile_threads"] == (threads or 512)
    for i, x in enumerate(insts):
        want = oracle.o1(x.seqs, x.n, x.m, x.l, x.d)[0]
        np.testing.assert_array_equal(got[i], want, err_msg="inst %d" % i)
        np.testing.assert_array_equal(alone[i], want, err_msg="inst %d" % i)


def test_batch_bad_instance_does_not_spoil_others():
    insts = mixed_instances(5, 6, [(9, 2), (10, 2)], (4, 8), (50, 120))
    bad = bytearray(insts[2].seqs)
    bad[7] = ord("x")
    items = [(x.seqs, x.n, x.m, x.l, x.d) for x in insts]
    items[2] = (bytes(bad), insts[2].n, insts[2].m, insts[2].l, insts[2].d)
    items.append((b"ACGT" * 3, 3, 4, 5, 1))            # l > m: EINVAL
    items.append((insts[0].seqs[:30 * 3], 3, 30, 30, 2))  # filter path alone
    with pms.Context() as c:
        got = c.solve_batch(items)
    assert isinstance(got[2], pms.PmsError) and got[2].status == pms.PMS_EBASE
    assert isinstance(got[6], pms.PmsError) and got[6].status == pms.PMS_EINVAL
    for i in (0, 1, 3, 4, 5, 7):
        s, n, m, l, d = items[i]
        np.testing.assert_array_equal(got[i], oracle.o1(s, n, m, l, d)[0])


def test_batch_large_output_retry():
    # two-letter strings give outputs far above the first heap estimate
    rng = random.Random(2)
    items = []
    for k in range(4):
        n, m, l, d = 3, 200, 9, 3
        s = bytes(rng.choice(b"AT") for _ in range(n * m))
        items.append((s, n, m, l, d))
    with pms.Context() as c:
        got = c.solve_batch(items)
        st = c.stats()
    for i, (s, n, m, l, d) in enumerate(items):
        np.testing.assert_array_equal(got[i], oracle.o1(s, n, m, l, d)[0])
    assert st["retries"] >= 1


@pytest.mark.parametrize("threads", [256, 512])
def test_served_tile_kernel_sizes(threads):
    # every serving launch on one forced workgroup size of the tile kernel
    reqs = mixed_instances(41, 12, [(9, 2), (13, 4)], (4, 8), (60, 150))
    say("served threads", threads)
    with pms.Context(serve_slots=4, tile_threads=threads) as c:
        tickets = [c.submit(x.seqs, x.n, x.m, x.l, x.d) for x in reqs]
        res = [c.wait(t, 60000) for t in tickets]
        for t in tickets:
            c.release(t)
    for i, x in enumerate(reqs):
        assert res[i] is not None
        np.testing.assert_array_equal(
            res[i], oracle.o1(x.seqs, x.n, x.m, x.l, x.d)[0],
            err_msg="request %d" % i)


def test_served_output_overflow_retries():
    # two-letter strings overflow the output room a request is first given
    # (about 6e4 motifs): the engine runs such a request again with room,
    # and the results still match the oracle and the same instance alone
    rng = random.Random(2)
    n, m, l, d = 3, 200, 9, 3
    items = [bytes(rng.choice(b"AT") for _ in range(n * m)) for _ in range(3)]
    small = mixed_instances(47, 6, [(9, 2), (11, 3)], (4, 10), (60, 200))
    with pms.Context(serve_slots=4) as c:
        tickets = [c.submit(x, n, m, l, d) for x in items]
        tickets += [c.submit(x.seqs, x.n, x.m, x.l, x.d) for x in small]
        res = [c.wait(t, 60000) for t in tickets]
        st = c.serve_stats()
        for t in tickets:
            c.release(t)
    assert st["retries"] >= 1
    for i, x in enumerate(items):
        np.testing.assert_array_equal(res[i], oracle.o1(x, n, m, l, d)[0])
    for i, x in enumerate(small):
        np.testing.assert_array_equal(
            res[len(items) + i], oracle.o1(x.seqs, x.n, x.m, x.l, x.d)[0])


def test_served_launch_size():
    # the launch size changes how requests share launches, never a result
    reqs = mixed_instances(43, 12, [(9, 2), (11, 3), (13, 4)], (4, 8),
                           (60, 150))
    want = [oracle.o1(x.seqs, x.n, x.m, x.l, x.d)[0] for x in reqs]
    for ms in (0.5, 32.0):
        say("served launch ms", ms)
        with pms.Context(serve_slots=4, serve_launch_ms=ms) as c:
            tickets = [c.submit(x.seqs, x.n, x.m, x.l, x.d) for x in reqs]
            res = [c.wait(t, 60000) for t in tickets]
            for t in tickets:
                c.release(t)
        for i in range(len(reqs)):
            assert res[i] is not None
            np.testing.assert_array_equal(res[i], want[i],
                                          err_msg="ms=%g request %d" % (ms, i))
    for bad in (-1.0, float("nan"), 5000.0):
        with pytest.raises(pms.PmsError):
            pms.Context(serve_launch_ms=bad)


def test_served_requests_match_alone_and_oracle():
    reqs = mixed_instances(33, 40, [(9, 2), (11, 3), (13, 4), (8, 1)],
                           (5, 20), (100, 600))
    with pms.Context(serve_slots=8) as c:
        tickets = []
        for i, x in enumerate(reqs):
            tickets.append(c.submit(x.seqs, x.n, x.m, x.l, x.d))
            if i % 7 == 0:
                time.sleep(0.002)   # arrivals while others run
        res = [c.wait(t, 60000) for t in tickets]
        times = [c.ticket_times(t) for t in tickets]
        st = c.serve_stats()
        for t in tickets:
            c.release(t)
        alone = [c.solve(x.seqs, x.n, x.m, x.l, x.d) for x in reqs]
    assert st["completed"] == len(reqs)
    assert st["max_inflight"] > 1          # requests overlapped on device
    for i, x in enumerate(reqs):
        assert res[i] is not None
        np.testing.assert_array_equal(res[i], alone[i])
        np.testing.assert_array_equal(
            res[i], oracle.o1(x.seqs, x.n, x.m, x.l, x.d)[0])
        ts, ta, td = times[i]
        assert ts <= ta <= td


def test_served_errors_and_queue_limit():
    x = pmsgen.planted(3, 6, 80, 9, 2)
    with pms.Context(serve_slots=1, serve_queue=2) as c:
        with pytest.raises(pms.PmsError) as e:
            c.submit(x.seqs, 6, 80, 9, 9)
        assert e.value.status == pms.PMS_EINVAL
        with pytest.raises(pms.PmsError) as e:
            c.submit(x.seqs[:6 * 40], 6, 40, 30, 2)   # 4^21 tiles: unsuitable
        assert e.value.status == pms.PMS_EINVAL
        bad = bytearray(x.seqs)
        bad[100] = ord("Z")
        tb = c.submit(bytes(bad), 6, 80, 9, 2)
        with pytest.raises(pms.PmsError) as e:
            c.wait(tb, 60000)
        assert e.value.status == pms.PMS_EBASE
        # flood a queue of 2 behind a single slot: some submits must bounce
        big = pmsgen.planted(4, 20, 600, 13, 4)
        busy = 0
        tickets = []
        for _ in range(40):
            try:
                tickets.append(c.submit(big.seqs, 20, 600, 13, 4))
            except pms.PmsError as err:
                assert err.status == pms.PMS_EBUSY
                busy += 1
        assert busy > 0
        want = oracle.o1(big.seqs, 20, 600, 13, 4)[0]
        for t in tickets:
            np.testing.assert_array_equal(c.wait(t, 120000), want)
        with pytest.raises(pms.PmsError):
            c.poll(999999)


def test_autotune_picks_a_valid_shape(tmp_path):
    cache = str(tmp_path / "tune.txt")
    x = pmsgen.planted(8, 10, 300, 11, 3)
    want = oracle.o1(x.seqs, 10, 300, 11, 3)[0]
    with pms.Context(tune_cache=cache) as c:
        s, t = c.autotune(10, 300, 11, 3)
        assert 3 <= s <= 9 and 1 <= t <= 256
        np.testing.assert_array_equal(c.solve(x.seqs, 10, 300, 11, 3), want)
        assert c.stats()["tile_suffix"] == s
        threads = c.stats()["tile_threads"]
    # one line "key s surv_t threads" (threads 0: chosen by tile size)
    fields = open(cache).read().split()
    assert len(fields) == 4 and (int(fields[1]), int(fields[2])) == (s, t)
    tpb = int(fields[3])
    assert tpb in (0, 256, 512)
    if tpb:
        assert threads == tpb
    # the cache file carries the choice to a new context
    with pms.Context(tune_cache=cache) as c2:
        np.testing.assert_array_equal(c2.solve(x.seqs, 10, 300, 11, 3), want)
        assert c2.stats()["tile_suffix"] == s
        assert c2.stats()["tile_threads"] == threads
