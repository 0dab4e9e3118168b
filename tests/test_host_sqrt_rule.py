"""The rounding rule behind the generator's radius square root, checked exhaustively on the host.

For a positive normal binary32 x and an estimate s within one ulp of sqrt(x), the correctly
rounded root is s- if x - s- s <= 0, s+ if x - s+ s > 0, and s otherwise (s-, s+ the neighbours
of s; the device evaluates the two differences with single-rounding fmas, whose signs are
exact).  Here the differences are formed exactly in binary64 (both terms are multiples of
ulp(s)^2 and differ by far fewer than 2^53 of them), and the rule is checked against numpy's
correctly rounded float32 square root for every x of three binades, each estimate s in
{RN(sqrt x) - 1 ulp, RN(sqrt x), RN(sqrt x) + 1 ulp}: [2^-24, 2^-23) holds the smallest
arguments the transform produces (about 1.2e-7), [1, 4) covers both exponent parities, and
[32, 64) the largest (33.3)."""
import numpy as np
import pytest


def rule(x: np.ndarray, s: np.ndarray) -> np.ndarray:
    sb = s.view(np.uint32)
    sm = (sb - np.uint32(1)).view(np.float32).astype(np.float64)
    sp = (sb + np.uint32(1)).view(np.float32).astype(np.float64)
    x64, s64 = x.astype(np.float64), s.astype(np.float64)
    r = np.where(x64 - sm * s64 <= 0, sm, s64)
    return np.where(x64 - sp * s64 > 0, sp, r).astype(np.float32)


@pytest.mark.parametrize("e0,e1", [(-24, -23), (0, 2), (5, 6)])
def test_rounding_rule_every_float_of_the_binades(e0, e1):
    for e in range(e0, e1):
        x = (np.uint32((e + 127) << 23) + np.arange(1 << 23, dtype=np.uint32)).view(np.float32)
        t = np.sqrt(x)
        tb = t.view(np.uint32)
        for d in (-1, 0, 1):
            s = (tb + np.uint32(d) if d >= 0 else tb - np.uint32(1)).view(np.float32)
            bad = np.count_nonzero(rule(x, s).view(np.uint32) != tb)
            assert bad == 0, (e, d, bad)


def test_rule_needs_both_neighbours():
    """An estimate one ulp low is only corrected by the upper test and one ulp high only by the
    lower test: a rule with either test missing gets those estimates wrong."""
    x = (np.uint32(127 << 23) + np.arange(1 << 20, dtype=np.uint32)).view(np.float32)
    t = np.sqrt(x)
    tb = t.view(np.uint32)
    below = (tb - np.uint32(1)).view(np.float32)
    above = (tb + np.uint32(1)).view(np.float32)
    assert np.array_equal(rule(x, below), t) and np.array_equal(rule(x, above), t)

    def lower_only(x, s):
        sm = (s.view(np.uint32) - np.uint32(1)).view(np.float32).astype(np.float64)
        return np.where(x.astype(np.float64) - sm * s.astype(np.float64) <= 0, sm, s).astype(np.float32)

    def upper_only(x, s):
        sp = (s.view(np.uint32) + np.uint32(1)).view(np.float32).astype(np.float64)
        return np.where(x.astype(np.float64) - sp * s.astype(np.float64) > 0, sp, s).astype(np.float32)

    assert not np.array_equal(lower_only(x, below), t)
    assert not np.array_equal(upper_only(x, above), t)
