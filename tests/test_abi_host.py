"""CPU checks of the C ABI library: it loads, exports every function include/dk_mlmc.h
declares, its struct sizes match the binding, and its host-side Algorithm 1 agrees exactly
with the oracle's on fake samplers (no GPU is touched)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import mlmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dk():
    import paper_2311_08872_amd as dk
    try:
        dk._lib.load()
    except RuntimeError as e:
        pytest.fail(f"library not built: {e}")
    return dk


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", fn)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*(dk_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol(dk):
    lib = C.CDLL(dk._lib.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    # the binding declares exactly the header's functions
    assert set(names) == set(dk._lib.SIGNATURES)


def test_version_and_error_string(dk):
    lib = dk._lib.load()
    assert b"gfx950" in lib.dk_version()
    assert lib.dk_last_error() is not None


def exact_sampler(means, sds):
    def sample(level, first, count):
        k = np.arange(first, first + count)
        return np.where(k % 2 == 0, 1.0, -1.0) * sds[level] + means[level]
    return sample


@pytest.mark.parametrize("eps", [5e-3, 2e-3, 1e-3])
def test_host_algorithm1_matches_oracle(dk, eps):
    L_max = 6
    means = [1.0] + [0.5 * 4.0 ** -l for l in range(1, L_max + 1)]
    sds = [1.0] + [0.5 * 2.0 ** -l for l in range(1, L_max + 1)]
    cost = [16.0 ** l * (1 + (l > 0) / 16) for l in range(L_max + 1)]
    s = exact_sampler(means, sds)
    lib_res = dk.alg1_host(eps, L_max, cost, s, m_pilot=1000)
    orc = mlmc.algorithm1(s, eps, L_max, lambda l: cost[l], M_bar=1000)
    assert lib_res["L"] == orc.L and lib_res["converged"] == orc.converged
    assert lib_res["M"] == orc.M
    assert np.allclose(lib_res["Yhat"], orc.Yhat, rtol=1e-12)
    assert np.allclose(lib_res["Vhat"], orc.Vhat, rtol=1e-9)
    assert abs(lib_res["estimate"][0] - orc.estimate) < 1e-12


def test_host_algorithm1_not_converged_and_errors(dk):
    means, sds = [1.0, 0.5, 0.5, 0.5], [1.0, 0.1, 0.1, 0.1]
    r = dk.alg1_host(1e-2, 3, [1, 16, 256, 4096], exact_sampler(means, sds), m_pilot=100)
    assert r["status"] == 1 and not r["converged"] and r["L"] == 3
    with pytest.raises(dk.DKError):
        dk.alg1_host(-1.0, 3, [1, 16, 256, 4096], exact_sampler(means, sds))
    with pytest.raises(dk.DKError):
        dk.alg1_host(1e-2, 3, [1, 0, 256, 4096], exact_sampler(means, sds))

    def nan_sampler(level, first, count):
        return np.full(count, np.nan)
    with pytest.raises(dk.DKError) as ei:
        dk.alg1_host(1e-2, 3, [1, 16, 256, 4096], nan_sampler)
    assert ei.value.code == -4

    def failing(level, first, count):
        raise ValueError("sampler failure")
    with pytest.raises(ValueError):
        dk.alg1_host(1e-2, 3, [1, 16, 256, 4096], failing)


def test_host_algorithm1_checkpoint_resume_is_bit_identical(dk, tmp_path):
    """A run killed inside a round resumes from its checkpoint and ends exactly where the
    uninterrupted run ends; the finished run's checkpoint reproduces the result without sampling;
    another run's file and a damaged file are rejected."""
    L_max = 5
    means = [1.0] + [0.5 * 4.0 ** -l for l in range(1, L_max + 1)]
    sds = [1.0] + [0.5 * 2.0 ** -l for l in range(1, L_max + 1)]
    cost = [16.0 ** l for l in range(L_max + 1)]
    s = exact_sampler(means, sds)
    full = dk.alg1_host(2e-3, L_max, cost, s, m_pilot=500)
    assert full["rounds"] >= 3
    path = tmp_path / "alg1.ckpt"
    calls = {"n": 0}

    def killed(level, first, count):
        calls["n"] += 1
        if calls["n"] == 7:
            raise RuntimeError("killed")
        return s(level, first, count)
    with pytest.raises(RuntimeError):
        dk.alg1_host(2e-3, L_max, cost, killed, m_pilot=500, checkpoint_path=path)
    assert path.exists()
    resumed = dk.alg1_host(2e-3, L_max, cost, s, m_pilot=500, checkpoint_path=path)
    for k in ("L", "converged", "rounds", "M", "Yhat", "Vhat", "estimate", "var_est", "rmse_est"):
        assert resumed[k] == full[k], k

    def never(level, first, count):
        raise AssertionError("a finished run must not sample again")
    again = dk.alg1_host(2e-3, L_max, cost, never, m_pilot=500, checkpoint_path=path)
    assert again["M"] == full["M"] and again["estimate"] == full["estimate"]
    with pytest.raises(dk.DKError):
        dk.alg1_host(1e-3, L_max, cost, s, m_pilot=500, checkpoint_path=path)     # another eps
    text = path.read_text()
    path.write_text(text[: len(text) // 2])
    with pytest.raises(dk.DKError):
        dk.alg1_host(2e-3, L_max, cost, s, m_pilot=500, checkpoint_path=path)
