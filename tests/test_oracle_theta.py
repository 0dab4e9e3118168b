"""Pins for the oracle's general-weight scheme (eq. (FullyDiscreteDK) with b0 > 0, b1 = 1 - b0;
``oracle.theta``): against facts that do not come from it.

* b0 = 0 is the explicit scheme, which the library oracle (C, a separate code path) runs;
* without noise every Fourier mode decays by (1 - 2 b1 mu s)/(1 + 2 b0 mu s) per step
  (Appendix A, operator A_h);
* the scheme conserves mass (both Lap_h and div_h sum to zero on the torus, and the solve
  keeps the mean);
* at high density E[P_l] = S_l and the NN pair variance of the linear observable equal the
  closed forms with A_h and the solve operator (the noise passes through the solve).
Statistical tolerances are 4.5 standard errors."""
import math

import numpy as np
import pytest

import dk_workloads as W
import oracle
from closed_forms import fluct_second_moment, heat_multiplier, pair_variance_linear
from oracle import theta

Z = 4.5


def test_b0_zero_is_the_explicit_scheme():
    p = W.config2(N=1e4)
    op = oracle.OracleProblem(p)
    for level, s in [(1, 3), (2, 11)]:
        a = theta.run_pair(p, level, s, cf=op.centre(level), cc=op.centre(level - 1))
        b = oracle.run_pair(op, level, s)
        assert np.max(np.abs(a - b)) <= 1e-10 * max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("b0", [0.5, 1.0])
def test_noise_free_mode_factor(b0):
    n, mu, steps = 16, 0.3, 37
    p = W.Problem(box=1.0, n0=n, levels=1, mu=mu, T=steps * mu / n ** 2, N=1e4, b0=b0,
                  rho0=W.Field(W.FIELD_MODES, 1.0, [W.Mode(0.5, 2, 3, 0.4)]))
    assert p.steps(0) == steps
    rho = theta.meanfield(p, 0)
    g = heat_multiplier(n, mu, b0)[3, 2]
    x = np.arange(n) / n
    X, Y = np.meshgrid(x, x)
    ref = 1.0 + 0.5 * g ** steps * np.cos(2 * math.pi * (2 * X + 3 * Y) + 0.4)
    assert np.max(np.abs(rho - ref)) < 1e-13


@pytest.mark.parametrize("b0", [0.5, 1.0])
def test_mass_is_conserved(b0):
    p = W.paper_reg(2e5).with_(b0=b0)
    P, rf, rc = theta.run_pair(p, 2, 5, want_field=True)
    for r, n in ((rf, p.n(2)), (rc, p.n(1))):
        r0 = oracle.field_grid(p.rho0, p.box, n)
        assert abs(r.sum() - r0.sum()) < 1e-12 * r0.sum()


@pytest.mark.parametrize("b0", [0.5, 1.0])
@pytest.mark.parametrize("level", [0, 1, 2])
def test_square_observable_mean_high_density(b0, level):
    p = W.paper_reg(2e9).with_(b0=b0)
    P = theta.run_range(p, level, 0, 2500, coupled=False)[:, 0, 0]
    S = fluct_second_moment(p, level, p.obs[0].phi)
    assert abs(P.mean() - S) < Z * P.std(ddof=1) / math.sqrt(len(P)), (P.mean(), S)


@pytest.mark.parametrize("b0", [0.5, 1.0])
@pytest.mark.parametrize("level,count", [(1, 2500), (2, 1200)])
def test_pair_variance_linear(b0, level, count):
    base = W.paper_reg(2e9).with_(b0=b0)
    phi = base.obs[0].phi
    p = base.with_(obs=[W.Obs(phi, True, True, W.PSI_ID)])
    P = theta.run_range(p, level, 0, count)
    Y = P[:, 0, 0] - P[:, 0, 1]
    V = pair_variance_linear(p, level, phi)
    assert abs(Y.mean()) < Z * Y.std(ddof=1) / math.sqrt(len(Y))
    assert abs(Y.var(ddof=1) / V - 1.0) < Z * math.sqrt(2.0 / len(Y)), (Y.var(ddof=1), V)
