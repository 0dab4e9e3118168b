"""The scheme of eq. (FullyDiscreteDK) with general weights b0 + b1 = 1 (test infrastructure only).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may use this module.  It shares no code with the HIP path.

One step solves, on the periodic grid,

    (I - tau b0/2 Lap_h) rho^m = (I + tau b1/2 Lap_h) rho^{m-1}
                                 + N^{-1/2} div_h( sqrt([rho^{m-1}]^+) h^{-d/2} Delta beta^{m-1} ),

with the 5-point Laplacian, the central divergence (Sec. 7) and d = 2.  The operator on the
left is diagonal in the discrete Fourier basis (eigenvalue 1 + tau b0/2 * 4/h^2 (sin^2(pi k1/n)
+ sin^2(pi k2/n))), so the solve is an FFT, a division and an inverse FFT (numpy, FP64).
b0 = 0 is the explicit Euler--Maruyama scheme of the other paths (Sec. 7).  Levels are coupled
as in Sec. 3.2 (NN coupling): the coarse increments are 2^{-d/2} times the fine ones summed over
the right-most 2 x 2 block and the 4 fine steps of a coarse step, and both grids take the same
scheme.
"""
from __future__ import annotations

import math

import numpy as np

import dk_workloads as W

from . import field_grid, noise_step


def laplacian(f: np.ndarray, h: float) -> np.ndarray:
    """5-point Laplacian on [y, x] arrays with periodic wrap."""
    return (np.roll(f, 1, 0) + np.roll(f, -1, 0) + np.roll(f, 1, 1) + np.roll(f, -1, 1) - 4.0 * f) / (h * h)


def theta_step(rho: np.ndarray, dbeta: np.ndarray, h: float, tau: float, N: float, b0: float) -> np.ndarray:
    """One step of eq. (FullyDiscreteDK); dbeta [y, x, r] are the Brownian increments."""
    n = rho.shape[0]
    b1 = 1.0 - b0
    amp = np.sqrt(np.maximum(rho, 0.0)) / h                  # sqrt([rho]^+) h^{-d/2}
    F0 = amp * dbeta[:, :, 0]                                # flux, direction x
    F1 = amp * dbeta[:, :, 1]                                # direction y
    div = (np.roll(F0, -1, 1) - np.roll(F0, 1, 1) + np.roll(F1, -1, 0) - np.roll(F1, 1, 0)) / (2.0 * h)
    rhs = rho + 0.5 * tau * b1 * laplacian(rho, h) + div / math.sqrt(N)
    s = np.sin(math.pi * np.arange(n) / n) ** 2
    eig = 1.0 + 0.5 * tau * b0 * 4.0 / (h * h) * (s[:, None] + s[None, :])
    return np.real(np.fft.ifft2(np.fft.fft2(rhs) / eig))


def _fields(p: W.Problem, n: int):
    return field_grid(p.rho0, p.box, n, p.offset), [field_grid(o.phi, p.box, n, p.offset) for o in p.obs]


def _observables(p: W.Problem, rho: np.ndarray, phis, n: int, centre: np.ndarray) -> np.ndarray:
    h2 = (p.box / n) ** 2
    P = np.zeros(len(p.obs))
    for j, o in enumerate(p.obs):
        L = h2 * float(np.sum(rho * phis[j]))
        X = (math.sqrt(p.N) if o.scale_sqrtN else 1.0) * (L - (centre[j] if o.centre else 0.0))
        P[j] = X * X if o.psi == W.PSI_SQUARE else X
    return P


def meanfield(p: W.Problem, level: int) -> np.ndarray:
    """rho_bar_l^M: the scheme without noise."""
    n, h, tau = p.n(level), p.h(level), p.tau(level)
    rho, _ = _fields(p, n)
    zero = np.zeros((n, n, 2))
    for _ in range(p.steps(level)):
        rho = theta_step(rho, zero, h, tau, p.N, p.b0)
    return rho


def centre(p: W.Problem, level: int) -> np.ndarray:
    n = p.n(level)
    rho = meanfield(p, level)
    _, phis = _fields(p, n)
    return np.array([(p.box / n) ** 2 * float(np.sum(rho * ph)) for ph in phis])


def run_single(p: W.Problem, level: int, sample: int, tag: int = W.TAG_MLMC, c: np.ndarray | None = None):
    n, h, tau = p.n(level), p.h(level), p.tau(level)
    c = centre(p, level) if c is None else c
    rho, phis = _fields(p, n)
    st = math.sqrt(tau)
    for m in range(p.steps(level)):
        z = noise_step(p.seed, tag, level, sample, n, m, f32=True).astype(np.float64)
        rho = theta_step(rho, st * z, h, tau, p.N, p.b0)
    return _observables(p, rho, phis, n, c)


def run_pair(p: W.Problem, level: int, sample: int, tag: int = W.TAG_MLMC, cf=None, cc=None, want_field=False):
    """(P_j^fine, P_j^coarse) of one NN-coupled pair with the scheme of weight b0 on both grids."""
    assert p.coupling == W.COUPLING_NN and level >= 1
    nf, nc = p.n(level), p.n(level - 1)
    hf, hc = p.h(level), p.h(level - 1)
    tf, tc = p.tau(level), p.tau(level - 1)
    cf = centre(p, level) if cf is None else cf
    cc = centre(p, level - 1) if cc is None else cc
    rf, phf = _fields(p, nf)
    rc, phc = _fields(p, nc)
    st = math.sqrt(tf)
    for mc in range(p.steps(level - 1)):
        Z = np.zeros((nc, nc, 2))
        for j in range(4):
            z = noise_step(p.seed, tag, level, sample, nf, 4 * mc + j, f32=True).astype(np.float64)
            rf = theta_step(rf, st * z, hf, tf, p.N, p.b0)
            Z += z[0::2, 0::2] + z[0::2, 1::2] + z[1::2, 0::2] + z[1::2, 1::2]
        rc = theta_step(rc, 0.5 * st * Z, hc, tc, p.N, p.b0)     # 2^{-d/2} sqrt(tau_f) Z
    P = np.stack([_observables(p, rf, phf, nf, cf), _observables(p, rc, phc, nc, cc)], axis=1)
    return (P, rf, rc) if want_field else P


def run_range(p: W.Problem, level: int, first: int, count: int, tag: int = W.TAG_MLMC,
              coupled: bool | None = None, threads: int = 8) -> np.ndarray:
    """Per-sample (P_fine, P_coarse) for samples [first, first + count): shape (count, n_obs, 2)."""
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
