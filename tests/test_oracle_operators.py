"""Pins for the oracle's EM step (eq. FullyDiscreteDK, b0 = 0, b1 = 1; Sec. 7 operators).

Brute force against dense matrices of the operators on 4x4 and 8x8 grids, the closed-form
spectrum of the 5-point Laplacian, summation by parts of the divergence against its
gradient partner, exact mass conservation, and the closed-form Fourier decay of the
noise-free scheme.
"""
import math

import numpy as np
import pytest

import dk_workloads as W
import oracle
from closed_forms import A_pow, field_np, grad, heat_multiplier


def dense_laplacian(n, h):
    """5-point Laplacian on the periodic n x n grid as an (n^2, n^2) matrix, site = x + n y."""
    L = np.zeros((n * n, n * n))
    for y in range(n):
        for x in range(n):
            s = x + n * y
            L[s, s] -= 4.0 / h ** 2
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                L[s, (x + dx) % n + n * ((y + dy) % n)] += 1.0 / h ** 2
    return L


def dense_divergence(n, h, flux):
    """Divergence as an (n^2, 2 n^2) matrix acting on b[site, r] flattened as 2*site + r."""
    D = np.zeros((n * n, 2 * n * n))
    for y in range(n):
        for x in range(n):
            s = x + n * y
            for r, (dx, dy) in enumerate(((1, 0), (0, 1))):
                plus = (x + dx) % n + n * ((y + dy) % n)
                minus = (x - dx) % n + n * ((y - dy) % n)
                if flux == W.FLUX_CENTRAL:
                    D[s, 2 * plus + r] += 1.0 / (2 * h)
                    D[s, 2 * minus + r] -= 1.0 / (2 * h)
                else:
                    D[s, 2 * s + r] += 1.0 / h
                    D[s, 2 * minus + r] -= 1.0 / h
    return D


def flux_field(rho, dbeta, h, flux):
    """[b]_r(y) = h^{-1} sqrt(m_r(y)^+) dbeta_{y,r} with m = rho (central) or the edge average."""
    n = rho.shape[0]
    b = np.zeros((n, n, 2))
    if flux == W.FLUX_CENTRAL:
        b[..., 0] = np.sqrt(np.maximum(rho, 0)) * dbeta[..., 0] / h
        b[..., 1] = np.sqrt(np.maximum(rho, 0)) * dbeta[..., 1] / h
    else:
        b[..., 0] = np.sqrt(np.maximum(0.5 * (rho + np.roll(rho, -1, 1)), 0)) * dbeta[..., 0] / h
        b[..., 1] = np.sqrt(np.maximum(0.5 * (rho + np.roll(rho, -1, 0)), 0)) * dbeta[..., 1] / h
    return b


@pytest.mark.parametrize("n", [4, 8])
@pytest.mark.parametrize("flux", [W.FLUX_CENTRAL, W.FLUX_STAGGERED])
def test_em_step_equals_dense_operator_form(n, flux):
    rng = np.random.default_rng(n + 10 * flux)
    h, tau, N = 1.0 / n, 0.1 / n ** 2, 37.0
    rho = 1.0 + 0.8 * rng.standard_normal((n, n))      # includes negative cells
    dbeta = math.sqrt(tau) * rng.standard_normal((n, n, 2))
    Lap = dense_laplacian(n, h)
    D = dense_divergence(n, h, flux)
    b = flux_field(rho, dbeta, h, flux).reshape(-1)
    expect = rho.reshape(-1) + 0.5 * tau * Lap @ rho.reshape(-1) + D @ b / math.sqrt(N)
    got = oracle.em_step(rho, dbeta, h, tau, N, flux).reshape(-1)
    assert np.max(np.abs(got - expect)) < 1e-12


@pytest.mark.parametrize("n", [4, 8])
def test_laplacian_spectrum(n):
    h = 1.0 / n
    ev = np.sort(np.linalg.eigvalsh(dense_laplacian(n, h)))
    k = np.arange(n)
    s = np.sin(math.pi * k / n) ** 2
    closed = np.sort((-(4.0 / h ** 2) * (s[None, :] + s[:, None])).ravel())
    assert np.allclose(ev, closed, rtol=0, atol=1e-9)


@pytest.mark.parametrize("flux", [W.FLUX_CENTRAL, W.FLUX_STAGGERED])
def test_divergence_summation_by_parts(flux):
    """(phi, div_h b)_h = -(grad_h phi, b)_h, with tau = 0 so that the step is rho + N^{-1/2} div b."""
    n, h, N = 16, 1.0 / 16, 1.0
    rng = np.random.default_rng(3)
    rho = 1.0 + 0.3 * rng.standard_normal((n, n))
    dbeta = rng.standard_normal((n, n, 2))
    divb = oracle.em_step(rho, dbeta, h, 0.0, N, flux) - rho
    phi = rng.standard_normal((n, n))
    b = flux_field(rho, dbeta, h, flux)
    gx, gy = grad(phi, h, flux)
    lhs = h * h * np.sum(phi * divb)
    rhs = -h * h * np.sum(gx * b[..., 0] + gy * b[..., 1])
    assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs))


@pytest.mark.parametrize("flux", [W.FLUX_CENTRAL, W.FLUX_STAGGERED])
def test_mass_conservation_over_many_steps(flux):
    n, h = 16, 1.0 / 16
    tau = 0.2 * h * h
    rng = np.random.default_rng(5)
    rho = 1.0 + 0.5 * rng.random((n, n))
    m0 = h * h * rho.sum()
    for m in range(300):
        dbeta = math.sqrt(tau) * rng.standard_normal((n, n, 2))
        rho = oracle.em_step(rho, dbeta, h, tau, 50.0, flux)   # low N: strong noise, negative cells
    assert (rho < 0).any()
    assert abs(h * h * rho.sum() - m0) < 4 * 300 * n * n * 2.0 ** -53 * np.abs(rho).max() * 10


def test_noise_free_fourier_decay_config1():
    """Config 1: <A^128 rho0, cos 2 pi x>_h = 0.25 g^128, g = 1 - 2 mu sin^2(pi/16)."""
    p = W.config1()
    op = oracle.OracleProblem(p)
    c, rho = oracle.meanfield(op, 0)
    g = 1.0 - 2.0 * 0.1 * math.sin(math.pi / 16) ** 2
    assert abs(g - 0.9923879532511287) < 1e-15
    assert abs(c[0] - 0.25 * g ** 128) < 1e-14
    assert abs(c[0] - 0.09400910494503552) < 1e-14


@pytest.mark.parametrize("level", [0, 1, 2])
def test_noise_free_decay_matches_fourier_multiplier(level):
    p = W.config2()
    op = oracle.OracleProblem(p)
    c, rho = oracle.meanfield(op, level)
    n = p.n(level)
    rho0 = field_np(p.rho0, p.box, n)
    expect = A_pow(rho0, p.steps(level), p.mu)
    assert np.max(np.abs(rho - expect)) < 1e-12
    # the single mode cos 2 pi x cos 2 pi y decays by g_{(1,1)}^M
    lam = heat_multiplier(n, p.mu)[1, 1]
    amp = 2 * np.mean(rho * np.cos(2 * math.pi * np.arange(n) / n)[None, :] *
                      np.cos(2 * math.pi * np.arange(n) / n)[:, None]) * 2
    assert abs(amp - 0.5 * lam ** p.steps(level)) < 1e-12
