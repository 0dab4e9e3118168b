"""Pins of the oracle's analytic fields that config 3 uses, against values the mathematics fixes
(no second transcription of the field formulas):

* the squared-bump observable's test function (a Gaussian bump of width sigma = 0.1 centred at
  (1/2, 1/2) with periodic minimum-image distance, amplitude 1): its grid sum h^2 sum phi equals
  the integral 2 pi sigma^2 erf(1 / (2 sqrt(2) sigma))^2 of the Gaussian over the unit torus (the
  trapezoid rule on a smooth periodic function converges faster than any power of h; the only
  non-smooth point, the minimum-image seam at distance 1/2, carries exp(-12.5) = 3.7e-6 of the
  peak), its second moment h^2 sum phi dx^2 equals sigma^2 times that, the sum is the same
  wherever the centre sits (a missing wrap loses most of the mass near a corner), and it peaks
  at 1 on the centre point;
* config 3's clipped initial datum max(0, cos 2 pi x) + 0.05: on an n x n grid with 4 | n its
  mean is cot(pi / n) / n + 0.05 exactly (the cosine sum over the nodes where it is positive is
  a geometric sum), it equals the floor 0.05 on the n/2 + 1 columns where cos 2 pi x <= 0 (up to
  the rounding of cos(pi / 2)), and its maximum is 1.05 at x = 0.
"""
import math

import numpy as np
import pytest

import dk_workloads as W
import oracle


def bump(sigma=0.1, cx=0.5, cy=0.5):
    return W.Field(W.FIELD_BUMP, 0.0, [], bump_amp=1.0, bump_sigma=sigma, bump_cx=cx, bump_cy=cy)


def test_config3_bump_is_the_workload_field():
    p = W.config3()
    f = p.obs[-1].phi
    assert f.kind == W.FIELD_BUMP and f.bump_sigma == 0.1 and (f.bump_cx, f.bump_cy) == (0.5, 0.5)
    assert f.bump_amp == 1.0 and f.c0 == 0.0
    assert p.obs[-1].psi == W.PSI_SQUARE and not p.obs[-1].centre and not p.obs[-1].scale_sqrtN


@pytest.mark.parametrize("n", [64, 128, 256])
@pytest.mark.parametrize("centre", [(0.5, 0.5), (0.05, 0.05), (0.0, 0.97), (0.3137, 0.8125)])
def test_bump_integral_and_second_moment(n, centre):
    sigma = 0.1
    g = oracle.field_grid(bump(sigma, *centre), 1.0, n)
    h = 1.0 / n
    exact = 2.0 * math.pi * sigma ** 2 * math.erf(1.0 / (2.0 * math.sqrt(2.0) * sigma)) ** 2
    assert abs(h * h * g.sum() / exact - 1.0) < 2e-6
    # second moment in x about the centre, with the periodic offset in [-1/2, 1/2)
    x = np.arange(n) * h
    dx = (x - centre[0] + 0.5) % 1.0 - 0.5
    m2 = h * h * float(np.sum(g * dx[None, :] ** 2))
    assert abs(m2 / (sigma ** 2 * exact) - 1.0) < 2e-4
    assert g.max() <= 1.0


@pytest.mark.parametrize("n", [8, 64, 256])
def test_bump_peak_on_the_centre_point(n):
    g = oracle.field_grid(bump(), 1.0, n)
    assert g[n // 2, n // 2] == 1.0
    assert np.unravel_index(np.argmax(g), g.shape) == (n // 2, n // 2)
    # mirror symmetry about the centre, including the points that wrap
    assert np.array_equal(g[:, 1:], g[:, 1:][:, ::-1])
    assert np.array_equal(g[1:, :], g[1:, :][::-1, :])


@pytest.mark.parametrize("n", [8, 16, 64, 256])
def test_clipped_datum_mean_floor_and_max(n):
    p = W.config3()
    g = oracle.field_grid(p.rho0, 1.0, n)
    assert g.shape == (n, n)
    mean = float(g.mean())
    assert abs(mean - (1.0 / (n * math.tan(math.pi / n)) + 0.05)) < 1e-14
    cols = g[0]
    floor_cols = np.sum(cols <= 0.05 + 1e-15)
    assert floor_cols == n // 2 + 1
    assert np.all(g == g[0:1, :])                       # independent of y
    assert cols[0] == 1.05 and cols.max() == 1.05
    assert np.all(cols >= 0.05)
