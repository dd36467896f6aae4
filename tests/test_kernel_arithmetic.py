"""Arithmetic facts the kernels rely on, checked on the CPU in FP32.

The first-order cross-overlap kernel splits a lane index x <= 64 (and the
wave width 64) by a molecule's atom count n <= 256 as
floor(x * rcp(n) + 2^-12), with rcp the hardware reciprocal (within one ulp
of 1/n) and the multiply-add rounded once.  This must equal x // n for every
such x and n, for any reciprocal within one ulp."""
import numpy as np


def test_reciprocal_division_is_exact():
    f = np.float32
    bad = []
    for n in range(1, 257):
        r = f(1.0) / f(n)
        for rr in (r, np.nextafter(r, f(0)), np.nextafter(r, f(2))):
            x = np.arange(0, 65, dtype=np.float64)
            # the fused multiply-add: exact product plus constant, rounded once
            q = (x * np.float64(rr) + 2.0 ** -12).astype(np.float32).astype(np.int64)
            wrong = np.nonzero(q != np.arange(0, 65) // n)[0]
            bad += [(n, int(w)) for w in wrong]
    assert not bad, bad[:10]
