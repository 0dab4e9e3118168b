"""Statistical pins for the oracle's sample paths, coupling and observables.

Each check follows from a statement of the paper (martingale lemma of Appendix A, the
equal-law remark of Sec. 3.1 that carries over to the NN coupling of Sec. 3.2, and the
cross-variation structure eq. (eqn:VarOfLvlPrelim)) and is evaluated in closed form by
``closed_forms`` (numpy, no oracle code).  Tolerances are 4.5 standard errors.
"""
import math

import numpy as np
import pytest
from scipy import stats

import dk_workloads as W
import oracle
from closed_forms import fluct_second_moment, linear_mean, one_step_sigma2, pair_variance_linear

Z = 4.5


def test_linear_mean_is_exact_config1():
    """E<rho^M, cos 2 pi x>_h = <A^M rho0, cos 2 pi x>_h = 0.0940091049... for every N."""
    p = W.config1()
    op = oracle.OracleProblem(p)
    P = oracle.run_range(op, 0, 0, 3000, tag=W.TAG_MC)[:, 0, 0]
    exact = linear_mean(p, 0, p.obs[0].phi)
    assert abs(exact - 0.09400910494503552) < 1e-14
    se = P.std(ddof=1) / math.sqrt(len(P))
    assert abs(P.mean() - exact) < Z * se
    # variance is bounded below by the mean-field value N^{-1} S (4.145e-4 for config 1)
    lin = W.Obs(p.obs[0].phi, True, True, W.PSI_ID)
    S = fluct_second_moment(p.with_(obs=[lin]), 0, lin.phi)
    assert abs(S / p.N - 4.145368e-4) < 1e-9
    var = P.var(ddof=1)
    assert var > S / p.N * (1 - Z * math.sqrt(2.0 / len(P)))


@pytest.mark.parametrize("flux", [W.FLUX_CENTRAL, W.FLUX_STAGGERED])
def test_one_step_law_is_gaussian(flux):
    """After one step from deterministic rho0, X = sqrt(N)(rho^1 - rho_bar^1, phi)_h ~ N(0, sigma^2),
    sigma^2 = tau (rho0^+, |grad_h phi|^2)_h exactly (any N)."""
    base = W.config2(N=300.0)
    phi = base.obs[0].phi
    p = base.with_(n0=8, levels=1, T=base.tau(0), flux=flux,
                   obs=[W.Obs(phi, True, True, W.PSI_ID), W.Obs(phi, True, True, W.PSI_SQUARE)])
    assert p.steps(0) == 1
    op = oracle.OracleProblem(p)
    P = oracle.run_range(op, 0, 0, 4000)
    X, X2 = P[:, 0, 0], P[:, 1, 0]
    s2 = one_step_sigma2(p, 0, phi)
    assert np.allclose(X * X, X2, rtol=1e-12, atol=1e-15)
    assert stats.kstest(X / math.sqrt(s2), "norm").pvalue > 1e-4
    assert abs(X2.mean() - s2) < Z * s2 * math.sqrt(2.0 / len(X2))


@pytest.mark.parametrize("level", [0, 1])
def test_square_observable_mean_high_density(level):
    """E[P_l] = S_l for psi = x^2 at high density (config 2 values 0.737003, 0.829074)."""
    p = W.config2(N=1e8)
    op = oracle.OracleProblem(p)
    P = oracle.run_range(op, level, 0, 3000, coupled=False)[:, 0, 0]
    S = fluct_second_moment(p, level, p.obs[0].phi)
    assert abs(S - [0.737003, 0.829074][level]) < 1e-6
    assert abs(P.mean() - S) < Z * P.std(ddof=1) / math.sqrt(len(P))


@pytest.mark.parametrize("flux", [W.FLUX_CENTRAL, W.FLUX_STAGGERED])
def test_pair_level_variance_high_density(flux):
    """Var(Y_1) of the linear centred observable equals the NN cross-variation formula
    (6.2571e-2 for config 2, pair 1, central)."""
    base = W.config2(N=1e8).with_(flux=flux)
    phi = base.obs[0].phi
    p = base.with_(obs=[W.Obs(phi, True, True, W.PSI_ID)])
    op = oracle.OracleProblem(p)
    P = oracle.run_range(op, 1, 0, 3000)
    Y = P[:, 0, 0] - P[:, 0, 1]
    V = pair_variance_linear(p, 1, phi)
    if flux == W.FLUX_CENTRAL:
        assert abs(V - 6.2571e-2) < 1e-6
    assert abs(Y.mean()) < Z * Y.std(ddof=1) / math.sqrt(len(Y))
    assert abs(Y.var(ddof=1) / V - 1.0) < Z * math.sqrt(2.0 / len(Y))


def test_restricted_noise_is_iid_standard_normal():
    """The coarse increments 2^{-d/2} sum_{B->, 4 steps} dbeta_f are i.i.d. N(0, tau_c)."""
    p = W.config2(N=1e4)
    op = oracle.OracleProblem(p)
    zs = np.stack([oracle.run_pair(op, 1, s, want_coarse_noise=True)[1] for s in range(600)])
    flat = zs.reshape(-1)
    assert abs(flat.mean()) < Z / math.sqrt(flat.size)
    assert abs(flat.var() - 1.0) < Z * math.sqrt(2.0 / flat.size)
    assert stats.kstest(flat, "norm").pvalue > 1e-4
    # no correlation between neighbouring coarse sites, nor between the two directions
    a = zs[:, :, :-1, 0].reshape(-1)
    b = zs[:, :, 1:, 0].reshape(-1)
    assert abs(np.corrcoef(a, b)[0, 1]) < Z / math.sqrt(a.size)
    assert abs(np.corrcoef(zs[..., 0].reshape(-1), zs[..., 1].reshape(-1))[0, 1]) < Z / math.sqrt(a.size)


def test_coarse_path_has_the_law_of_an_independent_path():
    """E and Var of P_{l-1} from the coarse member of pair l equal those of an uncoupled
    level-(l-1) path (equal-law remark of Sec. 3.1, stated for the NN coupling in Sec. 3.2)."""
    p = W.config2(N=1e4)
    op = oracle.OracleProblem(p)
    Pc = oracle.run_range(op, 1, 0, 4000)[:, 0, 1]
    P0 = oracle.run_range(op, 0, 0, 4000, coupled=False)[:, 0, 0]
    se = math.sqrt(Pc.var(ddof=1) / len(Pc) + P0.var(ddof=1) / len(P0))
    assert abs(Pc.mean() - P0.mean()) < Z * se
    f = Pc.var(ddof=1) / P0.var(ddof=1)
    lo, hi = stats.f.ppf([1e-5, 1 - 1e-5], len(Pc) - 1, len(P0) - 1)
    # P = X^2 is heavy-tailed; use a widened F interval
    assert lo * 0.8 < f < hi * 1.25
