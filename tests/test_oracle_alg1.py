"""Pins for the oracle's Algorithm 1 (Sec. 7) on fake level samplers with known statistics.

The samplers return exactly prescribed sample means and variances, so the optimal sample
counts of eq. (opt_M_ell) and the stopping level of eq. (convergence_criterion) are known in
closed form.
"""
import math

import numpy as np
import pytest

from oracle import mlmc


def exact_sampler(means, sds):
    """Values mean_l +- sd_l alternating in the sample index: after M draws the sample mean is
    mean_l (M even) or within sd_l / M of it, and the sample variance is sd_l^2 (1 + O(1/M))."""
    def sample(level, first, count):
        k = np.arange(first, first + count)
        return np.where(k % 2 == 0, 1.0, -1.0) * sds[level] + means[level]
    return sample


def test_optimal_M_formula():
    V = np.array([1.0, 0.25, 0.0625])
    Cst = np.array([1.0, 16.0, 256.0])
    eps = 1e-2
    s = sum(math.sqrt(v * c) for v, c in zip(V, Cst))
    expect = [math.ceil(2 * eps ** -2 * math.sqrt(v / c) * s) for v, c in zip(V, Cst)]
    assert list(mlmc.optimal_M(eps, V, Cst)) == expect


def test_convergence_criterion():
    eps = 1e-2
    thr = eps / math.sqrt(2) * 3.0   # (2^alpha - 1) = 3 for alpha = 2
    Y = np.array([1.0, 0.5 * thr, 0.9 * thr * 4, 0.9 * thr])
    assert mlmc.converged(Y, 3, eps)
    Y2 = Y.copy()
    Y2[1] = 16 * thr * 1.01           # 2^{-2 alpha} |Y_{L-2}| above the threshold
    assert not mlmc.converged(Y2, 3, eps)


def test_algorithm1_sample_counts_and_stopping_level():
    L_max = 6
    means = [1.0] + [0.5 * 4.0 ** -l for l in range(1, L_max + 1)]
    sds = [1.0] + [0.5 * 2.0 ** -l for l in range(1, L_max + 1)]     # V_l ~ 4^{-l}
    cost = lambda l: 16.0 ** l                                        # C_l ~ 2^{(d+2) l}
    eps = 2e-3
    res = mlmc.algorithm1(exact_sampler(means, [s for s in sds]), eps, L_max, cost, M_bar=1000)
    # the first L >= 2 that passes the bias test with these exact means
    L_expect = next(L for L in range(2, L_max + 1) if mlmc.converged(np.array(means), L, eps))
    assert res.converged and res.L == L_expect
    # final M_l satisfy eq. (opt_M_ell) for the final variance estimates, and are no larger
    # than the pilot size or the optimum for the exact variances (up to O(1/M) effects)
    Cst = np.array([cost(l) for l in range(res.L + 1)])
    M_hat = mlmc.optimal_M(eps, np.array(res.Vhat), Cst)
    M_true = mlmc.optimal_M(eps, np.array(sds[:res.L + 1]) ** 2, Cst)
    for l in range(res.L + 1):
        assert abs(res.Vhat[l] / sds[l] ** 2 - 1) < 2e-3
        assert res.M[l] >= M_hat[l]
        assert res.M[l] <= max(1000, int(M_true[l] * 1.002) + 2)
    assert res.var_est <= eps ** 2 / 2 * 1.001


def test_algorithm1_stops_at_L_max_without_convergence():
    L_max = 3
    means = [1.0, 0.5, 0.5, 0.5]      # no decay: the bias test never passes
    sds = [1.0, 0.1, 0.1, 0.1]
    res = mlmc.algorithm1(exact_sampler(means, sds), 1e-2, L_max, lambda l: 16.0 ** l, M_bar=100)
    assert not res.converged and res.L == L_max


def test_algorithm1_rmse_over_replicas():
    """Random (Gaussian) fake levels: the MLMC estimate's empirical RMSE is at most eps."""
    L_max = 6
    mu = [1.0] + [0.4 * 4.0 ** -l for l in range(1, L_max + 1)]
    sd = [1.0] + [0.6 * 2.0 ** -l for l in range(1, L_max + 1)]
    truth = sum(mu)
    eps = 1e-2
    errs = []
    for rep in range(60):
        rng = np.random.default_rng(rep)
        def sampler(level, first, count):
            return rng.normal(mu[level], sd[level], size=count)
        res = mlmc.algorithm1(sampler, eps, L_max, lambda l: 16.0 ** l, M_bar=200)
        errs.append(res.estimate - sum(mu[res.L + 1:]) * 0 - truth)
    rmse = math.sqrt(np.mean(np.square(errs)))
    assert rmse <= eps
