"""Problem statements and seeded synthetic workloads for the Dean--Kawasaki MLMC path.

This module only *describes* problems: grid hierarchy, CFL ratio, final time, particle
number, initial mean-field profile and test functions (Cornalba & Fischer, Sec. 2
definition of the discrete model, Sec. 3 observables, Sec. 7 setting).  It holds none of
the method's arithmetic: both the HIP path and the CPU oracle marshal these objects into
their own C structures.

Analytic fields on the torus [0, box)^2 (evaluated at grid points x_i = i*h, i.e. the
pointwise interpolation I_h of Sec. 2):

* ``FIELD_MODES``     f = c0 + sum_k amp_k cos(2 pi (kx_k x + ky_k y)/box + phase_k)
* ``FIELD_CLIPPED``   f = max(0, c0 + sum_k ...) + floor_add
* ``FIELD_BUMP``      f = c0 + bump_amp exp(-dist^2 / (2 sigma^2)), dist = periodic
                      minimum-image distance to (bump_cx, bump_cy)
* ``FIELD_EXPSIN2``   f = es_scale (es_a + es_b exp(-(sin^2(x-x0) + sin^2(y-y0))/(2 es_s)))
                      (the form of the paper's two Sec. 7 initial conditions)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List

import numpy as np

FIELD_MODES = 0
FIELD_CLIPPED = 1
FIELD_BUMP = 2
FIELD_EXPSIN2 = 3

PSI_ID = 0
PSI_SQUARE = 1

FLUX_CENTRAL = 0      # central difference of node fluxes (Sec. 7 operators)
FLUX_STAGGERED = 1    # forward difference of edge fluxes

STEPS_EXACT = 0       # T / tau_0 must be an integer
STEPS_ROUND_T = 1     # M_0 = round(T / tau_0); the effective final time is M_0 tau_0

PREC_F32 = 0
PREC_F64 = 1

GRID_VERTEX = 0        # grid points x_i = i h
GRID_CELL = 1          # cell centres x_i = (i + 1/2) h: the symmetric NN coupling (remark after Sec. 3.2)

COUPLING_NN = 0        # right-most nearest-neighbour coupling, h_(l-1) = 2 h_l (Sec. 3.2)
COUPLING_FOURIER = 1   # Fourier coupling, h_(l-1) = 3 h_l (Sec. 3.1)

TAG_MLMC = 0
TAG_MC = 1
TAG_CV_TRAIN = 2
TAG_CV_COARSE = 3


@dataclass
class Mode:
    amp: float
    kx: float
    ky: float
    phase: float = 0.0


@dataclass
class Field:
    kind: int = FIELD_MODES
    c0: float = 0.0
    modes: List[Mode] = field(default_factory=list)
    floor_add: float = 0.0
    bump_amp: float = 1.0
    bump_sigma: float = 0.1
    bump_cx: float = 0.5
    bump_cy: float = 0.5
    es_a: float = 1.0
    es_b: float = 0.0
    es_s: float = 1.0
    es_x0: float = 0.0
    es_y0: float = 0.0
    es_scale: float = 1.0


@dataclass
class Obs:
    phi: Field
    centre: bool = False        # subtract (rho_bar^M, I_h phi)_h of the discrete mean field
    scale_sqrtN: bool = False   # multiply by N^{1/2}
    psi: int = PSI_ID           # identity or square


@dataclass
class Problem:
    box: float = 1.0
    n0: int = 8
    levels: int = 1             # number of levels, L_max + 1
    mu: float = 0.1             # tau_l / h_l^2
    T: float = 0.05
    N: float = 1e4
    steps_policy: int = STEPS_EXACT
    flux: int = FLUX_CENTRAL
    precision: int = PREC_F32
    rho0: Field = field(default_factory=lambda: Field(c0=1.0))
    obs: List[Obs] = field(default_factory=list)
    primary: int = 0
    seed: int = 0
    coupling: int = COUPLING_NN
    grid: int = GRID_VERTEX
    b0: float = 0.0             # implicit weight of eq. (FullyDiscreteDK), b1 = 1 - b0 (0: explicit EM)

    # --- derived level data (pure bookkeeping, no method arithmetic) ---
    @property
    def ratio(self) -> int:
        """h_(l-1) / h_l: 2 for the NN coupling, 3 for the Fourier coupling (Sec. 3)."""
        return 3 if self.coupling == COUPLING_FOURIER else 2

    def n(self, level: int) -> int:
        return self.n0 * self.ratio ** level

    @property
    def offset(self) -> float:
        """Grid points are x_i = (i + offset) h."""
        return 0.5 if self.grid == GRID_CELL else 0.0

    def h(self, level: int) -> float:
        return self.box / self.n(level)

    def tau(self, level: int) -> float:
        return self.mu * self.h(level) ** 2

    def steps(self, level: int) -> int:
        m0 = self.T / self.tau(0)
        r = int(round(m0))
        if self.steps_policy == STEPS_EXACT and abs(m0 - r) > 1e-9 * max(1.0, r):
            raise ValueError(f"T/tau_0 = {m0} is not an integer")
        return r * self.ratio ** (2 * level)

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def cos_mode(k1: float, k2: float, amp: float = 1.0) -> Mode:
    return Mode(amp, k1, k2, 0.0)


def sin_mode(k1: float, k2: float, amp: float = 1.0) -> Mode:
    # sin(t) = cos(t - pi/2)
    return Mode(amp, k1, k2, -0.5 * math.pi)


# ----------------------------------------------------------------------------------------
# The five synthetic workloads.  Each returns a Problem.
# ----------------------------------------------------------------------------------------

def config1() -> Problem:
    """Plain single-level MC: 16x16 unit torus, rho0 = 1 + 0.5 cos(2 pi x), N = 1e3,
    tau = 0.1 h^2, T = 0.05 (128 steps), observable <rho_T, cos 2 pi x>_h (uncentred)."""
    return Problem(box=1.0, n0=16, levels=1, mu=0.1, T=0.05, N=1e3,
                   rho0=Field(FIELD_MODES, 1.0, [cos_mode(1, 0, 0.5)]),
                   obs=[Obs(Field(FIELD_MODES, 0.0, [cos_mode(1, 0)]), False, False, PSI_ID)],
                   primary=0, seed=0)


def config2_obs() -> List[Obs]:
    # primary: the paper's P with phi = sin 2 pi x + sin 2 pi y, psi = x^2, centred, sqrt(N) scaled
    primary = Obs(Field(FIELD_MODES, 0.0, [sin_mode(1, 0), sin_mode(0, 1)]), True, True, PSI_SQUARE)
    # secondary: uncentred linear <rho_T, cos 2 pi x cos 2 pi y>_h
    secondary = Obs(Field(FIELD_MODES, 0.0, [cos_mode(1, 1, 0.5), cos_mode(1, -1, 0.5)]),
                    False, False, PSI_ID)
    return [primary, secondary]


def config2(N: float = 1e4) -> Problem:
    """Plain MLMC: levels h = 1/8 .. 1/128, tau_l = 0.1 h_l^2, T = 0.05,
    rho0 = 1 + 0.5 cos 2 pi x cos 2 pi y, N = 1e4."""
    return Problem(box=1.0, n0=8, levels=5, mu=0.1, T=0.05, N=N,
                   rho0=Field(FIELD_MODES, 1.0, [cos_mode(1, 1, 0.25), cos_mode(1, -1, 0.25)]),
                   obs=config2_obs(), primary=0, seed=0)


def fourier_modes_k3():
    """Wave vectors with Euclidean |k| <= 3, k != 0, one of each +-k pair."""
    ks = []
    for k1 in range(0, 4):
        for k2 in range(-3, 4):
            if k1 * k1 + k2 * k2 == 0 or k1 * k1 + k2 * k2 > 9:
                continue
            if k1 == 0 and k2 <= 0:
                continue
            ks.append((k1, k2))
    return ks


def config3(N: float = 1e5) -> Problem:
    """Low-density MLMC: rho0 = max(0, cos 2 pi x) + 0.05, 6 levels h = 1/8 .. 1/256,
    observables: cos and sin parts of the Fourier modes |k| <= 3, plus <rho_T, bump>^2."""
    obs = []
    for (k1, k2) in fourier_modes_k3():
        obs.append(Obs(Field(FIELD_MODES, 0.0, [cos_mode(k1, k2)]), False, False, PSI_ID))
        obs.append(Obs(Field(FIELD_MODES, 0.0, [sin_mode(k1, k2)]), False, False, PSI_ID))
    obs.append(Obs(Field(FIELD_BUMP, 0.0, [], bump_amp=1.0, bump_sigma=0.1, bump_cx=0.5, bump_cy=0.5),
                   False, False, PSI_SQUARE))
    return Problem(box=1.0, n0=8, levels=6, mu=0.1, T=0.05, N=N,
                   rho0=Field(FIELD_CLIPPED, 0.0, [cos_mode(1, 0)], floor_add=0.05),
                   obs=obs, primary=len(obs) - 1, seed=0)


def config4() -> Problem:
    """Learned control variate workload: the config-2 settings."""
    return config2()


def random_modes(n_modes: int = 8, seed: int = 0, amp_max: float = 0.1, kmax: int = 8) -> List[Mode]:
    """Seeded random Fourier modes: k in {1..kmax}^2 with random signs, phase ~ U(0, 2 pi),
    amplitude ~ U(0, amp_max)."""
    rng = np.random.default_rng(seed)
    modes = []
    for _ in range(n_modes):
        k1 = int(rng.integers(1, kmax + 1)) * (1 if rng.random() < 0.5 else -1)
        k2 = int(rng.integers(1, kmax + 1)) * (1 if rng.random() < 0.5 else -1)
        modes.append(Mode(float(rng.uniform(0.0, amp_max)), float(k1), float(k2),
                          float(rng.uniform(0.0, 2.0 * math.pi))))
    return modes


def config5(N: float = 1e6) -> Problem:
    """Throughput scale: 7 levels h = 1/16 .. 1/1024, N = 1e6, tau = 0.1 h^2,
    T = 0.01 (rounded to a whole number of level-0 steps), rho0 = 1 + 8 random modes."""
    return Problem(box=1.0, n0=16, levels=7, mu=0.1, T=0.01, N=N, steps_policy=STEPS_ROUND_T,
                   rho0=Field(FIELD_MODES, 1.0, random_modes(8, 0)),
                   obs=config2_obs()[:1], primary=0, seed=0)


def _bessel_i0(x: float) -> float:
    """Modified Bessel function I_0 by its power series sum_k (x/2)^(2k) / (k!)^2."""
    term, total, k = 1.0, 1.0, 0
    while term > 1e-17 * total:
        k += 1
        term *= (x / 2.0) ** 2 / (k * k)
        total += term
    return total


def _expsin2_mass(a: float, b: float, s: float) -> float:
    """Integral over (0, 2 pi)^2 of a + b exp(-(sin^2(x - x0) + sin^2(y - y0)) / (2 s)): with
    sin^2 = (1 - cos 2x)/2 each axis gives 2 pi exp(-1/(4s)) I_0(1/(4s))."""
    two_pi = 2.0 * math.pi
    axis = two_pi * math.exp(-1.0 / (4.0 * s)) * _bessel_i0(1.0 / (4.0 * s))
    return a * two_pi * two_pi + b * axis * axis


def _paper_problem(N: float, a: float, b: float, s: float) -> Problem:
    """The paper's Sec. 7 setting: the 2 pi torus, h_l = 2 pi 2^-(2+l) (4 x 4 .. 128 x 128, six
    levels), tau_l = 1e-3 4^(5-l) (constant tau/h^2 = 1.024/(pi/2)^2 ~ 0.415), T = 1.024,
    phi = sin x + sin y, psi = x^2 of the centred, sqrt(N)-scaled observable, and the initial
    datum normalised to unit mass.  The state is FP64: at N = 2e9 the density of a fine cell
    fluctuates by ~1e-4 of itself, so binary32 rounding of the state alone would be ~1e-3 of the
    centred, sqrt(N)-scaled observable."""
    two_pi = 2.0 * math.pi
    h5 = two_pi / 128.0
    mu = 1e-3 / (h5 * h5)
    rho0 = Field(FIELD_EXPSIN2, es_a=a, es_b=b, es_s=s, es_x0=0.5 * math.pi, es_y0=1.5 * math.pi,
                 es_scale=1.0 / _expsin2_mass(a, b, s))
    phi = Field(FIELD_MODES, 0.0, [sin_mode(1, 0), sin_mode(0, 1)])
    return Problem(box=two_pi, n0=4, levels=6, mu=mu, T=1.024, N=N, steps_policy=STEPS_ROUND_T,
                   rho0=rho0, obs=[Obs(phi, True, True, PSI_SQUARE)], primary=0, seed=0, precision=PREC_F64)


def paper_reg(N: float = 2e9) -> Problem:
    """Sec. 7 with the regular datum Z^-1 (1 + exp(-(sin^2(x - pi/2) + sin^2(y - 3 pi/2))/2) / sqrt(2 pi))."""
    return _paper_problem(N, 1.0, 1.0 / math.sqrt(2.0 * math.pi), 1.0)


def paper_irreg(N: float = 2e9) -> Problem:
    """Sec. 7 with the irregular datum Z^-1 exp(-(sin^2(x - pi/2) + sin^2(y - 3 pi/2))/(2 * 0.1))."""
    return _paper_problem(N, 0.0, 1.0, 0.1)


def paper_fourier(N: float = 2e9, irregular: bool = False) -> Problem:
    """The Sec. 7 setting with the Fourier coupling of Sec. 3.1 instead of the NN coupling: the
    same torus, datum, observable, T and tau/h^2, but h_(l-1) = 3 h_l, so the hierarchy is
    4 x 4, 12 x 12, 36 x 36, 108 x 108 (1, 9, 81, 729 steps; h_min = 2 pi / 108, close to the
    NN hierarchy's 2 pi / 128)."""
    base = paper_irreg(N) if irregular else paper_reg(N)
    return base.with_(coupling=COUPLING_FOURIER, levels=4)
