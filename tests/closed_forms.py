"""Closed-form reference values for the discrete Dean--Kawasaki scheme (numpy, no oracle).

These are consequences of the paper's statements, computed in Fourier space, and serve as
pins for the oracle (they share no code with it):

* the noise-free scheme is rho^{m+1} = A rho^m with A = (I - tau b0/2 Lap_h)^{-1}(I + tau b1/2
  Lap_h) (Appendix A), whose Fourier multiplier is g_k = (1 - 2 b1 mu s_k)/(1 + 2 b0 mu s_k),
  s_k = sin^2(pi k1/n) + sin^2(pi k2/n) (b0 = 0, b1 = 1 is the explicit scheme of Sec. 7); the
  noise increment passes through (I - tau b0/2 Lap_h)^{-1} as well;
* Lemma "lem_Discrete_Martingale": (rho^m, A^{M-m} phi)_h is a martingale, hence
  E<rho^M, phi>_h = <A^M rho^0, phi>_h for every N (the noise increments have mean 0);
* the martingale increments are orthogonal, which gives
  E[X^2] = sum_m tau (E[rho^m]^+, |grad_h phi^{m+1}|^2)_h for X = sqrt(N)(rho^M - rho_bar^M, phi)_h
  (with equality to the mean-field value when rho stays positive);
* for the NN coupling of Sec. 3.2 the same computation on the pair gives the level
  variance of eq. (eqn:VarOfLvlPrelim) with rho replaced by the mean field;
* for the Fourier coupling of Sec. 3.1 the coarse noise is the fine noise projected onto the
  coarse frequencies (summed over the 9 fine steps) and read at the coarse nodes; the
  projection is written here in real space as a sum of cosines (restriction_1d), and the
  level variance follows as for the NN coupling with the lift replaced by its transpose.
"""
from __future__ import annotations

import math

import numpy as np

import dk_workloads as W


def grid(n: int, box: float, offset: float = 0.0):
    x = (np.arange(n) + offset) * (box / n)
    X, Y = np.meshgrid(x, x)      # arrays indexed [y, x]
    return X, Y


def field_np(f: W.Field, box: float, n: int, offset: float = 0.0) -> np.ndarray:
    X, Y = grid(n, box, offset)
    v = np.full((n, n), f.c0, dtype=np.float64)
    if f.kind in (W.FIELD_MODES, W.FIELD_CLIPPED):
        for m in f.modes:
            v = v + m.amp * np.cos(2 * math.pi * (m.kx * X + m.ky * Y) / box + m.phase)
        if f.kind == W.FIELD_CLIPPED:
            v = np.maximum(v, 0.0) + f.floor_add
        return v
    if f.kind == W.FIELD_BUMP:
        dx = np.abs(X - f.bump_cx) % box
        dx = np.minimum(dx, box - dx)
        dy = np.abs(Y - f.bump_cy) % box
        dy = np.minimum(dy, box - dy)
        return v + f.bump_amp * np.exp(-(dx * dx + dy * dy) / (2 * f.bump_sigma ** 2))
    if f.kind == W.FIELD_EXPSIN2:
        sx = np.sin(X - f.es_x0)
        sy = np.sin(Y - f.es_y0)
        return f.es_scale * (f.es_a + f.es_b * np.exp(-(sx * sx + sy * sy) / (2 * f.es_s)))
    raise ValueError(f.kind)


def heat_multiplier(n: int, mu: float, b0: float = 0.0) -> np.ndarray:
    """Fourier multiplier of the noise-free step A_h = (I - tau b0/2 Lap_h)^{-1} (I + tau b1/2 Lap_h)
    (Appendix A), b1 = 1 - b0: (1 - 2 b1 mu s) / (1 + 2 b0 mu s), s = sin^2(pi k1/n) + sin^2(pi k2/n)."""
    k = np.arange(n)
    s = np.sin(math.pi * k / n) ** 2
    ss = s[None, :] + s[:, None]
    return (1.0 - 2.0 * (1.0 - b0) * mu * ss) / (1.0 + 2.0 * b0 * mu * ss)


def solve_multiplier(n: int, mu: float, b0: float) -> np.ndarray:
    """Multiplier of (I - tau b0/2 Lap_h)^{-1}, which the noise increment also passes through."""
    k = np.arange(n)
    s = np.sin(math.pi * k / n) ** 2
    return 1.0 / (1.0 + 2.0 * b0 * mu * (s[None, :] + s[:, None]))


def A_pow(f: np.ndarray, m: int, mu: float, b0: float = 0.0) -> np.ndarray:
    lam = heat_multiplier(f.shape[0], mu, b0)
    return np.real(np.fft.ifft2(np.fft.fft2(f) * lam ** m))


def grad(f: np.ndarray, h: float, flux: int):
    """Adjoint partner of the divergence: central gradient for the central divergence,
    forward gradient for the staggered one.  Returns (d/dx, d/dy) on [y, x] arrays."""
    if flux == W.FLUX_CENTRAL:
        gx = (np.roll(f, -1, axis=1) - np.roll(f, 1, axis=1)) / (2 * h)
        gy = (np.roll(f, -1, axis=0) - np.roll(f, 1, axis=0)) / (2 * h)
    else:
        gx = (np.roll(f, -1, axis=1) - f) / h
        gy = (np.roll(f, -1, axis=0) - f) / h
    return gx, gy


def mobility(rho: np.ndarray, flux: int):
    """[rho]^+ where the noise of direction r is applied (node, or edge average)."""
    if flux == W.FLUX_CENTRAL:
        r = np.maximum(rho, 0.0)
        return r, r
    rx = np.maximum(0.5 * (rho + np.roll(rho, -1, axis=1)), 0.0)
    ry = np.maximum(0.5 * (rho + np.roll(rho, -1, axis=0)), 0.0)
    return rx, ry


def linear_mean(p: W.Problem, level: int, phi: W.Field) -> float:
    n, h = p.n(level), p.h(level)
    rho0 = field_np(p.rho0, p.box, n, p.offset)
    return float(h * h * np.sum(A_pow(rho0, p.steps(level), p.mu, p.b0) * field_np(phi, p.box, n, p.offset)))


def fluct_second_moment(p: W.Problem, level: int, phi: W.Field, flux: int | None = None) -> float:
    """S_l = sum_{m<M} tau (rho_bar^m, |grad_h phi^{m+1}|^2)_h : E[X^2] of the centred,
    sqrt(N)-scaled linear observable in the high-density limit (exact lower bound)."""
    flux = p.flux if flux is None else flux
    n, h, tau, M = p.n(level), p.h(level), p.tau(level), p.steps(level)
    lam = heat_multiplier(n, p.mu, p.b0)
    sol = solve_multiplier(n, p.mu, p.b0)
    r0 = np.fft.fft2(field_np(p.rho0, p.box, n, p.offset))
    f0 = np.fft.fft2(field_np(phi, p.box, n, p.offset))
    S = 0.0
    for m in range(M):
        rho = np.real(np.fft.ifft2(r0 * lam ** m))
        ph = np.real(np.fft.ifft2(f0 * sol * lam ** (M - m - 1)))
        gx, gy = grad(ph, h, flux)
        mx, my = mobility(rho, flux)
        S += tau * h * h * float(np.sum(mx * gx * gx + my * gy * gy))
    return S


def pair_variance_linear(p: W.Problem, level: int, phi: W.Field, flux: int | None = None) -> float:
    """Var(X_f - X_c) for the centred, sqrt(N)-scaled linear observable of the NN-coupled
    pair (fine level l, coarse l-1) in the high-density limit: the cross-variation
    structure of eq. (eqn:VarOfLvlPrelim) summed over fine steps.  Fine site y = (x, y)
    belongs to the coarse cell (x // 2, y // 2) (right-most block B->)."""
    flux = p.flux if flux is None else flux
    nf, nc = p.n(level), p.n(level - 1)
    hf, hc = p.h(level), p.h(level - 1)
    tf = p.tau(level)
    Mf = p.steps(level)
    Mc = Mf // 4
    lamf, lamc = heat_multiplier(nf, p.mu, p.b0), heat_multiplier(nc, p.mu, p.b0)
    solf, solc = solve_multiplier(nf, p.mu, p.b0), solve_multiplier(nc, p.mu, p.b0)
    rf0 = np.fft.fft2(field_np(p.rho0, p.box, nf, p.offset))
    rc0 = np.fft.fft2(field_np(p.rho0, p.box, nc, p.offset))
    ff0 = np.fft.fft2(field_np(phi, p.box, nf, p.offset))
    fc0 = np.fft.fft2(field_np(phi, p.box, nc, p.offset))
    V = 0.0
    coarse_cache = {}
    for m in range(Mf):
        mc = m // 4
        if mc not in coarse_cache:
            rc = np.real(np.fft.ifft2(rc0 * lamc ** mc))
            phc = np.real(np.fft.ifft2(fc0 * solc * lamc ** (Mc - mc - 1)))
            gcx, gcy = grad(phc, hc, flux)
            mcx, mcy = mobility(rc, flux)
            ax = np.sqrt(mcx) * gcx
            ay = np.sqrt(mcy) * gcy
            # lift to the fine grid: fine (x, y) -> coarse (x//2, y//2)
            coarse_cache = {mc: (np.kron(ax, np.ones((2, 2))), np.kron(ay, np.ones((2, 2))))}
        cx, cy = coarse_cache[mc]
        rf = np.real(np.fft.ifft2(rf0 * lamf ** m))
        phf = np.real(np.fft.ifft2(ff0 * solf * lamf ** (Mf - m - 1)))
        gfx, gfy = grad(phf, hf, flux)
        mfx, mfy = mobility(rf, flux)
        dx = np.sqrt(mfx) * gfx - cx
        dy = np.sqrt(mfy) * gfy - cy
        V += tf * hf * hf * float(np.sum(dx * dx + dy * dy))
    return V


def restriction_1d(nf: int, nc: int) -> np.ndarray:
    """Real-space kernel K[i_c, i] of the projection of a fine grid function onto the coarse
    frequencies {-nc/2, .., nc/2} (weight 2^{-1/2} on +-nc/2), read at coarse node 3 i_c:
    K = (1/nf) [1 + 2 sum_{k=1}^{nc/2-1} cos(2 pi k d / nf) + sqrt(2) cos(pi nc d / nf)],
    d = 3 i_c - i.  In 2-D the projection is K (x) K."""
    assert nf == 3 * nc and nc % 2 == 0
    d = 3 * np.arange(nc)[:, None] - np.arange(nf)[None, :]
    K = np.ones((nc, nf))
    for k in range(1, nc // 2):
        K += 2.0 * np.cos(2 * math.pi * k * d / nf)
    K += math.sqrt(2.0) * np.cos(math.pi * nc * d / nf)
    return K / nf


def pair_variance_linear_fourier(p: W.Problem, level: int, phi: W.Field) -> float:
    """Var(X_f - X_c) for the centred, sqrt(N)-scaled linear observable of the Fourier-coupled
    pair (h_c = 3 h_f, 9 fine steps per coarse step, central flux) in the high-density limit.
    X_f = -sum_{m,y,r} h_f sqrt(tau_f) g_f^m(y) z^m_r(y) with g = sqrt(rho_bar) grad phi (the
    adjoint form of the noise term); the coarse noise is h_f^{-1} sqrt(tau_f) (K x K) applied to
    the fine normals summed over the coarse step, so X_c has the coefficient
    h_f sqrt(tau_f) 9 (K x K)^T g_c on every fine normal of that step."""
    nf, nc = p.n(level), p.n(level - 1)
    hf, hc = p.h(level), p.h(level - 1)
    tf = p.tau(level)
    Mf = p.steps(level)
    Mc = Mf // 9
    K = restriction_1d(nf, nc)
    lamf, lamc = heat_multiplier(nf, p.mu), heat_multiplier(nc, p.mu)
    rf0 = np.fft.fft2(field_np(p.rho0, p.box, nf, p.offset))
    rc0 = np.fft.fft2(field_np(p.rho0, p.box, nc, p.offset))
    ff0 = np.fft.fft2(field_np(phi, p.box, nf, p.offset))
    fc0 = np.fft.fft2(field_np(phi, p.box, nc, p.offset))
    V = 0.0
    lifted = None
    for m in range(Mf):
        mc = m // 9
        if m % 9 == 0:
            rc = np.real(np.fft.ifft2(rc0 * lamc ** mc))
            phc = np.real(np.fft.ifft2(fc0 * lamc ** (Mc - mc - 1)))
            gcx, gcy = grad(phc, hc, W.FLUX_CENTRAL)
            sq = np.sqrt(np.maximum(rc, 0.0))
            # [y, x] arrays: (K x K)^T g = K^T g K
            lifted = (9.0 * K.T @ (sq * gcx) @ K, 9.0 * K.T @ (sq * gcy) @ K)
        rf = np.real(np.fft.ifft2(rf0 * lamf ** m))
        phf = np.real(np.fft.ifft2(ff0 * lamf ** (Mf - m - 1)))
        gfx, gfy = grad(phf, hf, W.FLUX_CENTRAL)
        sq = np.sqrt(np.maximum(rf, 0.0))
        dx = sq * gfx - lifted[0]
        dy = sq * gfy - lifted[1]
        V += tf * hf * hf * float(np.sum(dx * dx + dy * dy))
    return V


def one_step_sigma2(p: W.Problem, level: int, phi: W.Field, flux: int | None = None) -> float:
    """Variance of X after exactly one step from a deterministic rho0: tau (rho0^+, |grad phi|^2)_h."""
    flux = p.flux if flux is None else flux
    n, h, tau = p.n(level), p.h(level), p.tau(level)
    rho0 = field_np(p.rho0, p.box, n, p.offset)
    gx, gy = grad(field_np(phi, p.box, n, p.offset), h, flux)
    mx, my = mobility(rho0, flux)
    return tau * h * h * float(np.sum(mx * gx * gx + my * gy * gy))
