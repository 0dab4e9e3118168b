"""Plain-Python MLMC estimator and Algorithm 1 (test infrastructure only).

Follows Cornalba & Fischer, Sec. 4 eq. (MLMCEstimator) and Sec. 7 "Types of experiments":

* estimator  mu = M_0^{-1} sum P_0 + sum_{l>=1} M_l^{-1} sum (P_l - P_{l-1});
* optimal sample counts, eq. (opt_M_ell):
      M_l = ceil( 2 eps^{-2} sqrt(V_l / C_l) sum_k sqrt(V_k C_k) );
* convergence test, eq. (convergence_criterion):
      max_{j in {0,1,2}} 2^{-j alpha} |E[P_{L-j} - P_{L-j-1}]| / (2^alpha - 1) < eps / sqrt(2),
  where 2 is the refinement ratio h_{l-1}/h_l of the NN coupling; with the Fourier coupling
  (ratio 3) the same test uses 3 in place of 2 (the bias is assumed to fall by ratio^alpha
  per level);
* Algorithm 1: start with L = 2 and a target of M_bar samples on levels 0, 1, 2; while extra
  samples are needed, draw them, update V_l, recompute the optimal M_l and test convergence;
  if not converged, add a level with an initial target.

Readings where the paper's listing leaves details open (each one stated in the design
notes): the new level's initial target is M_bar; the convergence test is taken once a round
needs no extra samples; V_l is the unbiased sample variance; the cost C_l is the number of
cell updates of one sample of level l (fine plus coarse); at L_max without convergence the
run stops and reports that it did not converge.

``sampler(level, first, count)`` must return the per-sample values Y = P_l - P_{l-1} of the
primary observable (shape (count,)), for samples [first, first + count).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np


def cost_cell_updates(n0: int, steps0: int, level: int, d: int = 2) -> float:
    """Cell updates of one sample of level l: n_l^d M_l on the fine grid, plus the coarse
    grid of a pair (2^{-(d+2)} of that) for l >= 1."""
    n = n0 << level
    M = steps0 << (2 * level)
    c = float(n ** d) * float(M)
    if level >= 1:
        c *= 1.0 + 2.0 ** (-(d + 2))
    return c


def optimal_M(eps: float, V: np.ndarray, Cst: np.ndarray) -> np.ndarray:
    """Eq. (opt_M_ell)."""
    V = np.asarray(V, dtype=np.float64)
    Cst = np.asarray(Cst, dtype=np.float64)
    s = np.sum(np.sqrt(V * Cst))
    return np.ceil(2.0 * eps ** -2 * np.sqrt(V / Cst) * s).astype(np.int64)


def converged(Yhat: np.ndarray, L: int, eps: float, alpha: float = 2.0, ratio: float = 2.0) -> bool:
    """Eq. (convergence_criterion) on levels L, L-1, L-2."""
    return remainder(Yhat, L, alpha, ratio) < eps / math.sqrt(2.0)


def remainder(Yhat: np.ndarray, L: int, alpha: float = 2.0, ratio: float = 2.0) -> float:
    return max(ratio ** (-j * alpha) * abs(Yhat[L - j]) for j in range(3)) / (ratio ** alpha - 1.0)


@dataclass
class Alg1Result:
    estimate: float
    L: int
    converged: bool
    M: List[int]
    Yhat: List[float]
    Vhat: List[float]
    cost: List[float]
    var_est: float
    rounds: int
    history: List[dict] = field(default_factory=list)


def algorithm1(sampler: Callable[[int, int, int], np.ndarray], eps: float, L_max: int,
               cost: Callable[[int], float], M_bar: int = 1000, L_start: int = 2,
               alpha: float = 2.0, ratio: float = 2.0) -> Alg1Result:
    L = L_start
    done = [0] * (L_max + 1)
    s1 = [0.0] * (L_max + 1)
    s2 = [0.0] * (L_max + 1)
    target = [M_bar if l <= L else 0 for l in range(L_max + 1)]
    Cst = np.array([cost(l) for l in range(L_max + 1)], dtype=np.float64)
    rounds = 0
    history = []
    conv = False
    while True:
        extra = [max(0, target[l] - done[l]) for l in range(L + 1)]
        if sum(extra) == 0:
            Yhat = np.array([s1[l] / done[l] for l in range(L + 1)])
            if converged(Yhat, L, eps, alpha, ratio):
                conv = True
                break
            if L == L_max:
                conv = False
                break
            L += 1
            target[L] = M_bar
            continue
        rounds += 1
        for l in range(L + 1):
            if extra[l] > 0:
                y = np.asarray(sampler(l, done[l], extra[l]), dtype=np.float64)
                s1[l] += float(np.sum(y))
                s2[l] += float(np.sum(y * y))
                done[l] += extra[l]
        Yhat = np.array([s1[l] / done[l] for l in range(L + 1)])
        V = np.array([max(0.0, (s2[l] - done[l] * Yhat[l] ** 2) / (done[l] - 1)) for l in range(L + 1)])
        Mopt = optimal_M(eps, V, Cst[:L + 1])
        for l in range(L + 1):
            target[l] = max(done[l], int(Mopt[l]))
        history.append({"L": L, "done": list(done[:L + 1]), "target": list(target[:L + 1]),
                        "V": V.tolist(), "Y": Yhat.tolist()})
    Yhat = np.array([s1[l] / done[l] for l in range(L + 1)])
    V = np.array([max(0.0, (s2[l] - done[l] * Yhat[l] ** 2) / (done[l] - 1)) for l in range(L + 1)])
    return Alg1Result(float(np.sum(Yhat)), L, conv, done[:L + 1], Yhat.tolist(), V.tolist(),
                      Cst[:L + 1].tolist(), float(np.sum(V / np.array(done[:L + 1]))), rounds, history)


def mlmc_estimator(samples: List[np.ndarray]) -> float:
    """Eq. (MLMCEstimator): samples[l] holds the values of P_l - P_{l-1} (P_{-1} = 0)."""
    return float(sum(np.mean(np.asarray(s, dtype=np.float64)) for s in samples))
