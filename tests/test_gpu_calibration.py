"""The calibration entry point (pms_test_rate): the filter's Hamming-test mix
at full occupancy. Its rate must be positive and physically possible: at
3.75 VALU instructions per test (the compiled loop), no more than the
derived integer peak of 256 CUs x 64 lanes x 2.4 GHz (with 10% slack for
the clock)."""
import pytest

import paper_2403_00306_amd as pms

pytestmark = pytest.mark.gpu


def test_test_rate_is_physical():
    with pms.Context() as c:
        r1 = c.test_rate()
        r2 = c.test_rate()
    peak = 256 * 64 * 2.4e9
    for r in (r1, r2):
        assert r > 0
        assert r * 3.75 <= 1.1 * peak, r
    print("tests/s", r1, r2, "fraction of derived peak", r1 * 3.75 / peak,
          flush=True)


def test_lds_rate_is_physical():
    # single-bit LDS atomic ORs: at most one per bank (32) per clock per CU
    with pms.Context() as c:
        r = c.lds_rate()
    peak = 256 * 32 * 2.4e9
    assert 0 < r <= 1.1 * peak, r
    print("lds ORs/s", r, "lane ORs per CU clock", r / (256 * 2.4e9),
          flush=True)
