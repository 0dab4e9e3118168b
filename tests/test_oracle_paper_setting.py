"""Pins for the oracle in the paper's own Sec. 7 setting (the 2 pi torus, h_l = 2 pi 2^-(2+l)
from 4 x 4, tau_l = 1e-3 4^(5-l), T = 1.024, phi = sin x + sin y, psi = x^2), used by the
replication of its Type-1 experiment.

* Both initial data have unit mass: the periodic trapezoid rule on a fine grid is exact to
  rounding for these analytic periodic fields, so it checks the Bessel-function normalisation.
* On the 4 x 4 level (one step of tau_0 = T) the observable X = sqrt(N)(rho^1 - rho_bar^1, phi)_h
  is Gaussian with variance tau (rho0^+, |grad_h phi|^2)_h.
* At high density E[P_l] equals S_l of the cross-variation formula, and Var(Y_1) of the linear
  observable equals the NN pair formula (pair 1 couples 8 x 8 with the 4 x 4 grid).
Tolerances are 4.5 standard errors.
"""
import math

import numpy as np
import pytest
from scipy import stats

import dk_workloads as W
import oracle
from closed_forms import fluct_second_moment, one_step_sigma2, pair_variance_linear

Z = 4.5


@pytest.mark.parametrize("make", [W.paper_reg, W.paper_irreg])
def test_initial_data_have_unit_mass(make):
    p = make()
    for n in (256, 512):
        f = oracle.field_grid(p.rho0, p.box, n)
        assert abs(f.sum() * (p.box / n) ** 2 - 1.0) < 1e-12


def test_hierarchy_matches_the_paper():
    p = W.paper_reg()
    assert [p.n(l) for l in range(p.levels)] == [4, 8, 16, 32, 64, 128]
    assert [p.steps(l) for l in range(p.levels)] == [1, 4, 16, 64, 256, 1024]
    assert abs(p.tau(5) - 1e-3) < 1e-15 and abs(p.mu - 1.024 / (math.pi / 2) ** 2) < 1e-12


@pytest.mark.parametrize("make", [W.paper_reg, W.paper_irreg])
def test_one_step_law_on_the_4x4_level(make):
    base = make(N=2e5)
    phi = base.obs[0].phi
    p = base.with_(obs=[W.Obs(phi, True, True, W.PSI_ID)])
    assert p.steps(0) == 1
    X = oracle.run_range(oracle.OracleProblem(p), 0, 0, 4000, coupled=False)[:, 0, 0]
    s2 = one_step_sigma2(p, 0, phi)
    assert stats.kstest(X / math.sqrt(s2), "norm").pvalue > 1e-4


@pytest.mark.parametrize("level", [0, 1, 2])
def test_square_observable_mean_high_density(level):
    p = W.paper_reg(N=2e9)
    P = oracle.run_range(oracle.OracleProblem(p), level, 0, 3000, coupled=False)[:, 0, 0]
    S = fluct_second_moment(p, level, p.obs[0].phi)
    assert abs(P.mean() - S) < Z * P.std(ddof=1) / math.sqrt(len(P))


@pytest.mark.parametrize("make", [W.paper_reg, W.paper_irreg])
def test_pair_variance_with_the_4x4_coarse_grid(make):
    base = make(N=2e9)
    phi = base.obs[0].phi
    p = base.with_(obs=[W.Obs(phi, True, True, W.PSI_ID)])
    P = oracle.run_range(oracle.OracleProblem(p), 1, 0, 3000)
    Y = P[:, 0, 0] - P[:, 0, 1]
    V = pair_variance_linear(p, 1, phi)
    assert abs(Y.mean()) < Z * Y.std(ddof=1) / math.sqrt(len(Y))
    assert abs(Y.var(ddof=1) / V - 1.0) < Z * math.sqrt(2.0 / len(Y))
