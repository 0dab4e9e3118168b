"""GPU parity of the general-weight scheme (b0 > 0 in eq. (FullyDiscreteDK)) against the FP64
oracle (``oracle.theta``, numpy FFT solves of the full system): per-sample observables in the
paper's Sec. 7 setting (FP64 state, the derived bound of the NN parity tests) for Crank--Nicolson
(b0 = 1/2) and implicit Euler (b0 = 1), config 2 with the FP32 state (1e-5 of the batch RMS),
a time step beyond the explicit limit with b0 = 1, Algorithm 1 against the oracle's, and the
argument checks."""
import math

import numpy as np
import pytest

import dk_workloads as W
import oracle
from oracle import mlmc, theta

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


def paper_theta(b0, N=2e9):
    return W.paper_reg(N).with_(b0=b0, levels=5)          # 4 .. 64


@pytest.mark.parametrize("b0", [0.5, 1.0])
@pytest.mark.parametrize("level,count", [(0, 200), (1, 100), (2, 50), (3, 20), (4, 6)])
def test_paper_setting_theta_parity(b0, level, count):
    p = paper_theta(b0)
    banner(f"b0={b0} paper setting level={level} n={p.n(level)} steps={p.steps(level)} count={count}")
    _, ps = dk.level_pair(p, level, 0, count, per_sample=True)
    torch.cuda.synchronize()
    ref = theta.run_range(p, level, 0, count)
    err = scaled_err(ps.cpu().numpy(), ref)
    n = p.n(level)
    rho0 = oracle.field_grid(p.rho0, p.box, n)
    phi = oracle.field_grid(p.obs[0].phi, p.box, n)
    terms = math.sqrt(p.N) * (p.box / n) ** 2 * float(np.sum(np.abs(rho0 * phi)))
    rms_x = math.sqrt(float(np.mean(ref[:, 0, 0])))
    tol = 64 * 1.1e-16 * terms / rms_x * math.sqrt(p.steps(level) + 1)
    banner(f"scaled FP64 error {err:.3g} (tolerance {tol:.3g})")
    assert err <= tol


@pytest.mark.parametrize("level,count", [(0, 100), (1, 60), (2, 24), (3, 6)])
def test_config2_theta_fp32_parity(level, count):
    p = W.config2(N=1e4).with_(b0=0.5, levels=4)
    banner(f"config2 b0=0.5 FP32 level={level} count={count}")
    _, ps = dk.level_pair(p, level, 3, count, per_sample=True)
    torch.cuda.synchronize()
    ref = theta.run_range(p, level, 3, count)
    err = scaled_err(ps.cpu().numpy(), ref)
    banner(f"scaled FP32-vs-FP64 error {err:.3g} (tolerance 1e-5)")
    assert err <= 1e-5


def test_cell_centred_crank_nicolson():
    """b0 = 1/2 on cell-centred grid points (the symmetric NN coupling): the two options compose."""
    p = W.config2(N=1e4).with_(b0=0.5, levels=4, grid=W.GRID_CELL)
    banner("b0=0.5 on cell centres, level 2")
    _, ps = dk.level_pair(p, 2, 0, 24, per_sample=True)
    torch.cuda.synchronize()
    ref = theta.run_range(p, 2, 0, 24)
    err = scaled_err(ps.cpu().numpy(), ref)
    banner(f"scaled FP32-vs-FP64 error {err:.3g} (tolerance 1e-5)")
    assert err <= 1e-5


def test_large_time_step_implicit_euler():
    """b0 = 1 with tau = 2 h^2 (four times the explicit limit mu <= 1/2), T = 2 tau_0."""
    p = W.config2(N=1e4).with_(b0=1.0, levels=4, mu=2.0, T=0.0625)
    assert p.steps(2) == 32
    banner("b0=1, mu=2")
    _, ps = dk.level_pair(p, 2, 0, 30, per_sample=True)
    torch.cuda.synchronize()
    ref = theta.run_range(p, 2, 0, 30)
    err = scaled_err(ps.cpu().numpy(), ref)
    banner(f"scaled FP32-vs-FP64 error {err:.3g} (tolerance 1e-5)")
    assert err <= 1e-5


def test_theta_algorithm1_matches_the_oracle():
    p = paper_theta(0.5)
    eps = 10 ** -1.4
    g = dk.estimate(p, eps)

    def sampler(level, first, count):
        P = theta.run_range(p, level, first, count)
        return P[:, 0, 0] - P[:, 0, 1]

    def cost(level):
        return p.n(level) ** 2 * p.steps(level) * (1.0 + (level > 0) / 16.0)

    o = mlmc.algorithm1(sampler, eps, p.levels - 1, cost, M_bar=1000)
    banner(f"GPU L={g['L']} M={g['M']} est={g['estimate'][0]:.6g}; oracle L={o.L} M={o.M} est={o.estimate:.6g}")
    assert g["L"] == o.L and list(g["M"]) == list(o.M[:o.L + 1])
    assert abs(g["estimate"][0] - o.estimate) <= 1e-9 * abs(o.estimate)


def test_theta_rejections():
    p = W.config2(N=1e4).with_(levels=4)
    with pytest.raises(dk.DKError):
        dk.level_pair(p.with_(b0=0.2, mu=1.0), 1, 0, 4)              # mu (1 - 2 b0) > 1/2
    with pytest.raises(dk.DKError):
        dk.level_pair(p.with_(b0=0.5, flux=W.FLUX_STAGGERED), 1, 0, 4)
    with pytest.raises(dk.DKError):
        dk.level_pair(W.config2(N=1e4).with_(b0=0.5), 1, 0, 4)       # 128 x 128 level
    with pytest.raises(dk.DKError):
        dk.level_pair(p.with_(b0=1.5), 1, 0, 4)
