"""GPU parity of the Fourier coupling (Sec. 3.1) against the FP64 oracle (``oracle.fourier``):
per-sample observables of single paths and pairs on every level of the paper's Sec. 7
setting with the Fourier hierarchy (4, 12, 36, 108; FP64 state, tolerance derived as for the
NN pairs in that setting) and of a unit-box hierarchy with the FP32 state (8, 24, 72; 1e-5 of
the batch RMS), Algorithm 1 against the oracle's at a loose accuracy, and argument checks."""
import math

import numpy as np
import pytest

import dk_workloads as W
from oracle import fourier as F
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


def unit_box_fourier(N=1e4):
    """Config-2 settings (unit torus, rho0 = 1 + 0.5 cos 2 pi x cos 2 pi y, tau = 0.1 h^2,
    T = 0.05, FP32) on the Fourier hierarchy 8, 24, 72 (32, 288, 2592 steps)."""
    return W.config2(N=N).with_(coupling=W.COUPLING_FOURIER, levels=3)


@pytest.mark.parametrize("N", [2e9, 2e5])
@pytest.mark.parametrize("level,count", [(0, 200), (1, 120), (2, 40), (3, 4)])
def test_paper_setting_fourier_parity(N, level, count):
    p = W.paper_fourier(N)
    banner(f"Fourier paper setting N={N:g} level={level} n={p.n(level)} steps={p.steps(level)} count={count}")
    _, ps = dk.level_pair(p, level, 0, count, per_sample=True)
    torch.cuda.synchronize()
    gpu = ps.cpu().numpy()
    ref = F.run_range(p, level, 0, count)
    err = scaled_err(gpu, ref)
    # FP64 bound as for the NN pairs of this setting: the centred observable cancels terms of
    # size sqrt(N) h^2 sum |rho phi|, each rounded to u = 1.1e-16, accumulated over the steps
    n = p.n(level)
    import oracle
    rho0 = oracle.field_grid(p.rho0, p.box, n)
    phi = oracle.field_grid(p.obs[0].phi, p.box, n)
    terms = math.sqrt(p.N) * (p.box / n) ** 2 * float(np.sum(np.abs(rho0 * phi)))
    rms_x = math.sqrt(float(np.mean(ref[:, 0, 0])))
    tol = 64 * 1.1e-16 * terms / rms_x * math.sqrt(p.steps(level) + 1)
    banner(f"scaled FP64 error {err:.3g} (tolerance {tol:.3g})")
    assert err <= tol
    if level >= 1:
        assert np.all(np.isfinite(gpu[:, 0, 1])) and np.any(gpu[:, 0, 1] != 0.0)


@pytest.mark.parametrize("level,count", [(0, 64), (1, 24), (2, 3)])
def test_unit_box_fourier_fp32_parity(level, count):
    p = unit_box_fourier()
    banner(f"Fourier unit box FP32 level={level} n={p.n(level)} steps={p.steps(level)} count={count}")
    _, ps = dk.level_pair(p, level, 5, count, per_sample=True)
    torch.cuda.synchronize()
    gpu = ps.cpu().numpy()
    ref = F.run_range(p, level, 5, count)
    err = scaled_err(gpu, ref)
    banner(f"scaled FP32-vs-FP64 error {err:.3g} (tolerance 1e-5)")
    assert err <= 1e-5


def test_fourier_batching_and_plain_mc():
    """Values do not depend on how a range is split into launches; plain-MC paths (tag 1) of a
    Fourier level are the oracle's single paths."""
    p = W.paper_fourier(2e9)
    _, whole = dk.level_pair(p, 2, 100, 50, per_sample=True)
    _, a = dk.level_pair(p, 2, 100, 17, per_sample=True)
    _, b = dk.level_pair(p, 2, 117, 33, per_sample=True)
    torch.cuda.synchronize()
    assert torch.equal(whole, torch.cat([a, b]))
    _, mc = dk.mc_level(p, 2, 0, 10, per_sample=True)
    torch.cuda.synchronize()
    ref = F.run_range(p, 2, 0, 10, tag=W.TAG_MC, coupled=False)
    assert np.allclose(mc.cpu().numpy()[:, :, 0], ref[:, :, 0], rtol=1e-9, atol=1e-12)


def test_fourier_algorithm1_matches_the_oracle():
    p = W.paper_fourier(2e9).with_(levels=3)
    eps = 10 ** -1.4
    banner(f"Fourier Algorithm 1, eps={eps:.3g}: GPU")
    g = dk.estimate(p, eps)

    def sampler(level, first, count):
        P = F.run_range(p, level, first, count)
        return P[:, 0, 0] - P[:, 0, 1]

    def cost(level):
        return p.n(level) ** 2 * p.steps(level) * (1.0 + (level > 0) / 81.0)

    banner("Fourier Algorithm 1: oracle")
    o = mlmc.algorithm1(sampler, eps, p.levels - 1, cost, M_bar=1000, ratio=3.0)
    banner(f"GPU L={g['L']} M={g['M']} est={g['estimate'][0]:.6g}; oracle L={o.L} M={o.M} est={o.estimate:.6g}")
    assert g["L"] == o.L and g["converged"] == o.converged
    assert list(g["M"]) == list(o.M[:o.L + 1])
    assert abs(g["estimate"][0] - o.estimate) <= 1e-9 * abs(o.estimate)


def test_fourier_rejections():
    p = W.paper_fourier(2e9)
    with pytest.raises(dk.DKError):
        dk.level_pair(p.with_(flux=W.FLUX_STAGGERED), 1, 0, 4)     # central flux only
    with pytest.raises(dk.DKError):
        dk.level_pair(p.with_(n0=6), 1, 0, 4)                       # no 18 x 18 kernel
    with pytest.raises(dk.DKError):
        dk.level_pair(p.with_(levels=5), 1, 0, 4)                   # 324 x 324 is beyond the kernel
