"""End-to-end parity in the paper's own Sec. 7 setting (2 pi torus, 4 x 4 .. 128 x 128,
tau_l = 1e-3 4^(5-l), T = 1.024, phi = sin x + sin y, psi = x^2): the library's Algorithm 1 on
the GPU (FP64 state, as this setting needs) and the oracle's Algorithm 1 (plain Python driving
the FP64 oracle) run the same sample indices of the same noise, so they choose the same levels
and sample counts, and their estimates agree to FP64 rounding.
"""
import pytest

import dk_workloads as W
import oracle
from oracle import mlmc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2311_08872_amd as dk  # noqa: E402


@pytest.mark.parametrize("make,N", [(W.paper_reg, 2e9), (W.paper_irreg, 2e9), (W.paper_reg, 2e5)])
def test_algorithm1_matches_the_oracle_at_the_loosest_accuracy(make, N):
    p = make(N)
    eps = 10 ** -1.4
    print(f"[gpu] {make.__name__} N={N:g} eps={eps:.3g}: GPU Algorithm 1", flush=True)
    g = dk.estimate(p, eps)
    op = oracle.OracleProblem(p)

    def sampler(level, first, count):
        P = oracle.run_range(op, level, first, count)
        return P[:, 0, 0] - P[:, 0, 1]

    def cost(level):
        return p.n(level) ** 2 * p.steps(level) * (1.0 + (level > 0) / 16.0)

    print(f"[gpu] {make.__name__} N={N:g}: oracle Algorithm 1", flush=True)
    o = mlmc.algorithm1(sampler, eps, p.levels - 1, cost, M_bar=1000)
    print(f"[gpu] GPU L={g['L']} M={g['M']} est={g['estimate'][0]:.6g}; oracle L={o.L} M={o.M} est={o.estimate:.6g}",
          flush=True)
    assert g["L"] == o.L and g["converged"] == o.converged
    assert list(g["M"]) == list(o.M[:o.L + 1])
    assert abs(g["estimate"][0] - o.estimate) <= 1e-9 * abs(o.estimate)
