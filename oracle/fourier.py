"""Fourier coupling of Sec. 3.1 in FP64 (test infrastructure only).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may use this module.  It shares no code with the HIP path.

Sec. 3.1 couples levels l-1 and l with h_{l-1} = 3 h_l and tau_{l-1} = 9 tau_l.  The noise of
level l is written in the orthonormal Fourier basis e_xi(x) = box^{-1} exp(2 pi i xi.x / box)
of the grid functions (inner product (f, g)_h = h^2 sum f conj(g)) over the frequencies
I_l = {-n_l/2, ..., n_l/2 - 1}^2 with complex Brownian motions (conjugate pairs, real ones at
the self-conjugate frequencies); the coarse level reuses the coefficients of the frequencies
it resolves, summed over the 9 fine steps of one coarse step.

* Fine noise.  The nodal increments Delta beta_x = sqrt(tau_l) z_x of the scheme (z i.i.d.
  N(0, 1), the same generator as every other level) give the field W(x) = h^{-1} Delta beta_x,
  whose Fourier coefficients (W, e_xi)_h are exactly such a family of Brownian increments (the
  orthonormal change of basis maps i.i.d. real Gaussians to independent conjugate pairs plus
  real self-conjugate coefficients, each of variance tau_l).  So the fine level of a Fourier
  pair runs the same nodal noise as the NN pair and the single-level path.
* Coarse noise.  W_c(x) = sum_{xi in I_{l-1}} e_xi(x) C_xi at the coarse nodes, with C_xi the
  coefficient of the fine noise summed over the 9 steps.  Reading (the paper leaves it open):
  a coarse frequency with a component -n_{l-1}/2 is the coarse grid's Nyquist frequency, on
  which e_xi and e_xi' coincide for xi' with that component +n_{l-1}/2; the fine grid resolves
  both, so C_xi is the sum over these aliases, times 2^{-1/2} per Nyquist component.  This is
  the choice for which W_c is real and has the law of the coarse level's own noise (i.i.d.
  nodal increments of variance tau_{l-1} h_{l-1}^{-2}); both facts are pinned in the tests.
* The coarse EM step then takes Delta beta~_x = h_{l-1} W_c(x).

Grid points are x = (i h, j h), i, j = 0 .. n-1 (the vertex grid), so every coarse node is a
fine node.
"""
from __future__ import annotations

import math

import numpy as np

import dk_workloads as W

from . import em_step, field_grid, noise_step


def coarse_increment(dbeta_sum: np.ndarray, box: float, nf: int, nc: int) -> np.ndarray:
    """Coarse nodal increments h_c W_c (shape (nc, nc, 2), [y, x, r]) from the fine nodal
    increments summed over the 9 fine steps of one coarse step (shape (nf, nf, 2))."""
    assert nf == 3 * nc and nc % 2 == 0
    hf, hc = box / nf, box / nc
    out = np.zeros((nc, nc, 2))
    half = nc // 2
    for r in range(2):
        Wsum = dbeta_sum[:, :, r] / hf                     # summed fine noise field W
        # (W, e_xi)_h = h^2 box^{-1} sum_x W(x) exp(-2 pi i xi.x / box), xi.x / box = k.i / nf
        coef = hf * hf / box * np.fft.fft2(Wsum)           # indexed [ky mod nf, kx mod nf]
        C = np.zeros((nc, nc), dtype=complex)              # coarse coefficients, [ky mod nc, kx mod nc]
        for ky in range(-half, half):
            for kx in range(-half, half):
                ys = [ky, half] if ky == -half else [ky]
                xs = [kx, half] if kx == -half else [kx]
                wgt = (2 ** -0.5 if ky == -half else 1.0) * (2 ** -0.5 if kx == -half else 1.0)
                C[ky % nc, kx % nc] = wgt * sum(coef[a % nf, b % nf] for a in ys for b in xs)
        # W_c(x_c) = sum_xi e_xi(x_c) C_xi = box^{-1} sum_k C_k exp(2 pi i k.j / nc)
        Wc = nc * nc / box * np.fft.ifft2(C)
        assert np.max(np.abs(Wc.imag)) <= 1e-9 * max(1.0, np.max(np.abs(Wc.real)))
        out[:, :, r] = hc * Wc.real
    return out


def _vertex(p: W.Problem):
    assert p.grid == W.GRID_VERTEX, "the Fourier coupling is set up on the vertex grid"


def _observables(p: W.Problem, rho: np.ndarray, n: int, centre: np.ndarray) -> np.ndarray:
    """P_j = psi_j(s_j ((rho, I_h phi_j)_h - c_j)) of eq. (eqn_MLMCLevels)."""
    h2 = (p.box / n) ** 2
    P = np.zeros(len(p.obs))
    for j, o in enumerate(p.obs):
        L = h2 * float(np.sum(rho * field_grid(o.phi, p.box, n)))
        X = (math.sqrt(p.N) if o.scale_sqrtN else 1.0) * (L - (centre[j] if o.centre else 0.0))
        P[j] = X * X if o.psi == W.PSI_SQUARE else X
    return P


def centre(p: W.Problem, level: int) -> np.ndarray:
    """c_{l,j} = (rho_bar_l^M, I_h phi_j)_h: the noise-free scheme run to the final time."""
    _vertex(p)
    n, h, tau = p.n(level), p.h(level), p.tau(level)
    rho = field_grid(p.rho0, p.box, n)
    zero = np.zeros((n, n, 2))
    for _ in range(p.steps(level)):
        rho = em_step(rho, zero, h, tau, p.N, p.flux)
    return np.array([(p.box / n) ** 2 * float(np.sum(rho * field_grid(o.phi, p.box, n))) for o in p.obs])


def run_single(p: W.Problem, level: int, sample: int, tag: int = W.TAG_MLMC, c: np.ndarray | None = None):
    """(P_j) of one uncoupled path on level `level` (level 0 of the estimator, or plain MC)."""
    _vertex(p)
    n, h, tau = p.n(level), p.h(level), p.tau(level)
    c = centre(p, level) if c is None else c
    rho = field_grid(p.rho0, p.box, n)
    st = math.sqrt(tau)
    for m in range(p.steps(level)):
        z = noise_step(p.seed, tag, level, sample, n, m, f32=True).astype(np.float64)
        rho = em_step(rho, st * z, h, tau, p.N, p.flux)
    return _observables(p, rho, n, c)


def run_pair(p: W.Problem, level: int, sample: int, tag: int = W.TAG_MLMC, cf: np.ndarray | None = None,
             cc: np.ndarray | None = None, want_field: bool = False):
    """(P_j^fine, P_j^coarse) of one Fourier-coupled pair (fine level `level`)."""
    assert p.coupling == W.COUPLING_FOURIER and level >= 1
    _vertex(p)
    nf, nc = p.n(level), p.n(level - 1)
    hf, hc = p.h(level), p.h(level - 1)
    tf, tc = p.tau(level), p.tau(level - 1)
    cf = centre(p, level) if cf is None else cf
    cc = centre(p, level - 1) if cc is None else cc
    rf = field_grid(p.rho0, p.box, nf)
    rc = field_grid(p.rho0, p.box, nc)
    st = math.sqrt(tf)
    for mc in range(p.steps(level - 1)):
        dsum = np.zeros((nf, nf, 2))
        for j in range(9):
            z = noise_step(p.seed, tag, level, sample, nf, 9 * mc + j, f32=True).astype(np.float64)
            rf = em_step(rf, st * z, hf, tf, p.N, p.flux)
            dsum += st * z
        rc = em_step(rc, coarse_increment(dsum, p.box, nf, nc), hc, tc, p.N, p.flux)
    P = np.stack([_observables(p, rf, nf, cf), _observables(p, rc, nc, cc)], axis=1)
    return (P, rf, rc) if want_field else P


def run_range(p: W.Problem, level: int, first: int, count: int, tag: int = W.TAG_MLMC,
              coupled: bool | None = None, threads: int = 8) -> np.ndarray:
    """Per-sample (P_fine, P_coarse) for samples [first, first + count): shape (count, n_obs, 2);
    the coarse column is zero for single paths."""
    from concurrent.futures import ThreadPoolExecutor
    if coupled is None:
        coupled = level >= 1
    cf = centre(p, level)
    cc = centre(p, level - 1) if coupled else None
    out = np.zeros((count, len(p.obs), 2))

    def one(i):
        if coupled:
            out[i] = run_pair(p, level, first + i, tag, cf, cc)
        else:
            out[i, :, 0] = run_single(p, level, first + i, tag, cf)

    with ThreadPoolExecutor(max(1, min(threads, count))) as ex:
        list(ex.map(one, range(count)))
    return out
