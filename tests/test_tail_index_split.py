"""CPU check of the index split used by the single-workgroup tail kernels.

The tail kernels (levels of at most 17^3 nodes, at most 65 per dimension)
split a node index t into (i, j, k) with quotients t / e computed as
trunc((t + 0.5) * rcp(e)) in single precision, rcp being the hardware
reciprocal (about one unit in the last place).  The claim: for 0 <= t < 2^13
and 1 <= e <= 65 this equals the integer quotient, because (t + 0.5) / e lies
at least 0.5 / e from an integer while the rounding error of the product
stays far smaller.  Checked here for every index and extent, with the
reciprocal correctly rounded and one unit off in either direction.
"""
import numpy as np


def test_single_precision_reciprocal_quotient_is_exact():
    t = np.arange(0, 1 << 13, dtype=np.int64)
    tf = t.astype(np.float32) + np.float32(0.5)
    for e in range(1, 66):
        r = np.float32(1.0) / np.float32(e)
        for rr in (np.nextafter(r, np.float32(0)), r, np.nextafter(r, np.float32(2))):
            q = (tf * rr).astype(np.float32).astype(np.int64)
            assert np.array_equal(q, t // e), e


def test_the_index_range_covers_the_tail_limits():
    # the largest tail level grid (kTailNodes = 17^3) and extent (65) stay
    # inside the checked range
    assert 17 ** 3 < (1 << 13)
    assert 65 * 65 < (1 << 13)
