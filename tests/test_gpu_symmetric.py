"""GPU parity of the symmetric NN coupling (cell-centred grid points, the remark after Sec. 3.2)
against the FP64 oracle: per-sample observables of config 2 (FP32 state, 1e-5 of the batch
RMS) and of the paper's Sec. 7 setting (FP64 state, the derived bound of the NN parity tests),
Algorithm 1 against the oracle's, and the rejection of the Fourier coupling on this grid."""
import math

import numpy as np
import pytest

import dk_workloads as W
import oracle
from oracle import mlmc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2311_08872_amd as dk  # noqa: E402


def banner(msg):
    print(f"[gpu] {msg}", flush=True)


def scaled_err(gpu, ref):
    rms = np.sqrt(np.mean(ref ** 2, axis=0, keepdims=True))
    return float(np.max(np.abs(gpu - ref) / np.maximum(np.maximum(np.abs(ref), rms), 1e-300)))


@pytest.mark.parametrize("level,count", [(0, 200), (1, 150), (2, 70), (3, 16)])
def test_config2_cell_centred_parity(level, count):
    p = W.config2(N=1e4).with_(grid=W.GRID_CELL)
    banner(f"config2 cell-centred level={level} count={count}")
    _, ps = dk.level_pair(p, level, 0, count, per_sample=True)
    torch.cuda.synchronize()
    ref = oracle.run_range(oracle.OracleProblem(p), level, 0, count)
    err = scaled_err(ps.cpu().numpy(), ref)
    banner(f"scaled FP32-vs-FP64 error {err:.3g} (tolerance 1e-5)")
    assert err <= 1e-5
    # the grid moved: the vertex-grid run of the same samples differs
    _, pv = dk.level_pair(p.with_(grid=W.GRID_VERTEX), level, 0, count, per_sample=True)
    torch.cuda.synchronize()
    assert not torch.equal(ps, pv)


@pytest.mark.parametrize("level,count", [(0, 300), (1, 200), (2, 100), (3, 40)])
def test_paper_setting_cell_centred_parity(level, count):
    p = W.paper_reg(2e9).with_(grid=W.GRID_CELL)
    banner(f"paper setting cell-centred level={level} count={count}")
    _, ps = dk.level_pair(p, level, 0, count, per_sample=True)
    torch.cuda.synchronize()
    ref = oracle.run_range(oracle.OracleProblem(p), level, 0, count)
    err = scaled_err(ps.cpu().numpy(), ref)
    n = p.n(level)
    rho0 = oracle.field_grid(p.rho0, p.box, n, 0.5)
    phi = oracle.field_grid(p.obs[0].phi, p.box, n, 0.5)
    terms = math.sqrt(p.N) * (p.box / n) ** 2 * float(np.sum(np.abs(rho0 * phi)))
    rms_x = math.sqrt(float(np.mean(ref[:, 0, 0])))
    tol = 64 * 1.1e-16 * terms / rms_x * math.sqrt(p.steps(level) + 1)
    banner(f"scaled FP64 error {err:.3g} (tolerance {tol:.3g})")
    assert err <= tol


def test_cell_centred_algorithm1_matches_the_oracle():
    p = W.paper_reg(2e9).with_(grid=W.GRID_CELL)
    eps = 10 ** -1.4
    banner(f"cell-centred Algorithm 1, eps={eps:.3g}")
    g = dk.estimate(p, eps)
    op = oracle.OracleProblem(p)

    def sampler(level, first, count):
        P = oracle.run_range(op, level, first, count)
        return P[:, 0, 0] - P[:, 0, 1]

    def cost(level):
        return p.n(level) ** 2 * p.steps(level) * (1.0 + (level > 0) / 16.0)

    o = mlmc.algorithm1(sampler, eps, p.levels - 1, cost, M_bar=1000)
    banner(f"GPU L={g['L']} M={g['M']} est={g['estimate'][0]:.6g}; oracle L={o.L} M={o.M} est={o.estimate:.6g}")
    assert g["L"] == o.L and list(g["M"]) == list(o.M[:o.L + 1])
    assert abs(g["estimate"][0] - o.estimate) <= 1e-9 * abs(o.estimate)


def test_fourier_on_cell_centres_is_rejected():
    with pytest.raises(dk.DKError):
        dk.level_pair(W.paper_fourier(2e9).with_(grid=W.GRID_CELL), 1, 0, 4)
