"""Pins for the oracle's Fourier coupling (Sec. 3.1; h_(l-1) = 3 h_l, 9 fine steps per coarse
step), checked against facts that do not come from the oracle:

* the coarse increments are a real, isometric image of the summed fine increments (M M^T = I),
  which is the statement that each level's noise has the law of that level's own noise
  (Remark distribution_W_ell): i.i.d. N(0, tau_(l-1)) nodal increments;
* the map equals the real-space projection kernel (sum of cosines, written independently in
  ``closed_forms.restriction_1d``), keeps band-limited fields (|k| < n_c/2) and removes the
  frequencies the coarse grid does not resolve;
* at high density, E[P_f] and E[P_c] of the Fourier pair equal the mean-field values S_l,
  S_(l-1) (each level's noise has its own level's law), and the pair variance of the linear
  observable equals the closed form of ``closed_forms.pair_variance_linear_fourier``.
Statistical tolerances are 4.5 standard errors.
"""
import math

import numpy as np
import pytest

import dk_workloads as W
from closed_forms import fluct_second_moment, pair_variance_linear_fourier, restriction_1d
from oracle import fourier as F

Z = 4.5


def _matrix(nf, nc, box, r):
    M = np.zeros((nc * nc, nf * nf))
    for i in range(nf * nf):
        d = np.zeros((nf, nf, 2))
        d.reshape(-1, 2)[i, r] = 1.0
        out = F.coarse_increment(d, box, nf, nc)
        assert np.all(out[:, :, 1 - r] == 0.0)
        M[:, i] = out[:, :, r].ravel()
    return M


@pytest.mark.parametrize("nf,nc", [(12, 4), (36, 12)])
@pytest.mark.parametrize("r", [0, 1])
def test_coarse_map_is_an_isometry_equal_to_the_projection_kernel(nf, nc, r):
    M = _matrix(nf, nc, 2 * math.pi, r)
    assert np.max(np.abs(M @ M.T - np.eye(nc * nc))) < 1e-12
    K = restriction_1d(nf, nc)
    assert np.max(np.abs(M - 3.0 * np.kron(K, K))) < 1e-12


@pytest.mark.parametrize("box", [1.0, 2 * math.pi])
def test_band_limited_fields(box):
    nf, nc = 36, 12
    i = np.arange(nf)
    X, Y = np.meshgrid(i, i)       # [y, x]

    def wave(kx, ky, ph=0.3):
        return np.cos(2 * math.pi * (kx * X + ky * Y) / nf + ph)

    for (kx, ky) in [(1, 0), (2, -3), (5, 5), (-4, 1)]:          # |k_i| < nc/2 = 6: kept
        d = np.stack([wave(kx, ky), wave(ky, kx, 1.1)], axis=-1)
        out = F.coarse_increment(d, box, nf, nc)
        assert np.max(np.abs(out - 3.0 * d[::3, ::3])) < 1e-12
    for (kx, ky) in [(7, 0), (0, 10), (8, 13), (17, 2)]:          # a component beyond 6: removed
        d = np.stack([wave(kx, ky), wave(kx, ky, 0.7)], axis=-1)
        assert np.max(np.abs(F.coarse_increment(d, box, nf, nc))) < 1e-12
    # the coarse Nyquist frequency keeps 2^{-1/2} of its amplitude per Nyquist component
    d = np.stack([wave(6, 0, 0.0), wave(6, 6, 0.0)], axis=-1)
    out = F.coarse_increment(d, box, nf, nc)
    assert np.max(np.abs(out[:, :, 0] - 3.0 / math.sqrt(2) * d[::3, ::3, 0])) < 1e-12
    assert np.max(np.abs(out[:, :, 1] - 1.5 * d[::3, ::3, 1])) < 1e-12


def test_coarse_increments_have_the_coarse_law():
    """Summed fine increments of 9 steps -> coarse increments with variance tau_c = 9 tau_f,
    uncorrelated between nodes (empirical, 4000 draws on 12 x 12 -> 4 x 4)."""
    rng = np.random.default_rng(5)
    nf, nc, tf = 12, 4, 0.01
    draws = np.stack([F.coarse_increment(math.sqrt(tf) * rng.standard_normal((9, nf, nf, 2)).sum(0),
                                         2 * math.pi, nf, nc).ravel() for _ in range(4000)])
    C = np.cov(draws.T) / (9 * tf)
    se = math.sqrt(2.0 / 4000)
    assert np.max(np.abs(np.diag(C) - 1.0)) < Z * se
    off = C - np.diag(np.diag(C))
    assert np.max(np.abs(off)) < Z * math.sqrt(1.0 / 4000) * 1.3


def _linear(p):
    phi = p.obs[0].phi
    return p.with_(obs=[W.Obs(phi, True, True, W.PSI_ID)]), phi


@pytest.mark.parametrize("level,count", [(1, 3000), (2, 400)])
def test_fourier_pair_means_at_high_density(level, count):
    p = W.paper_fourier(N=2e9)
    P = F.run_range(p, level, 0, count)[:, 0, :]
    for col, lv in ((0, level), (1, level - 1)):
        S = fluct_second_moment(p, lv, p.obs[0].phi)
        x = P[:, col]
        assert abs(x.mean() - S) < Z * x.std(ddof=1) / math.sqrt(count), (lv, x.mean(), S)


@pytest.mark.parametrize("level,count", [(1, 3000), (2, 400)])
def test_fourier_pair_variance_of_the_linear_observable(level, count):
    p, phi = _linear(W.paper_fourier(N=2e9))
    P = F.run_range(p, level, 0, count)[:, 0, :]
    Y = P[:, 0] - P[:, 1]
    V = pair_variance_linear_fourier(p, level, phi)
    assert abs(Y.mean()) < Z * Y.std(ddof=1) / math.sqrt(count)
    assert abs(Y.var(ddof=1) / V - 1.0) < Z * math.sqrt(2.0 / count), (Y.var(ddof=1), V)


def test_single_level_matches_the_pair_fine_member():
    """The fine member of a Fourier pair and the single-level path of the same level and
    sample use the same noise, so they end in the same field."""
    p = W.paper_fourier(N=2e5)
    P, rf, rc = F.run_pair(p, 2, 7, want_field=True)
    assert abs(F.run_single(p, 2, 7)[0] - P[0, 0]) <= 1e-12 * abs(P[0, 0])
