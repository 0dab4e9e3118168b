"""Power of the oracle's pins: plausible mistakes planted in a copy of the oracle (on the CPU)
must each fail at least one pin.

Each mutant is a text substitution in oracle/dk_oracle.c compiled into a temporary library;
the test swaps it in, runs the pin that should catch it, expects that pin to fail, and restores
the regular build.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import dk_workloads as W
import oracle
from closed_forms import A_pow, field_np, one_step_sigma2, pair_variance_linear

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "dk_oracle.c")


def build_mutant(old: str, new: str) -> str:
    src = open(SRC).read()
    assert src.count(old) >= 1, old
    d = tempfile.mkdtemp(prefix="dk_mutant_")
    c = os.path.join(d, "m.c")
    so = os.path.join(d, "libm.so")
    open(c, "w").write(src.replace(old, new, 1))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-o", so, c, "-lm"])
    return so


@pytest.fixture
def mutant():
    libs = []

    def use(old, new):
        so = build_mutant(old, new)
        libs.append(so)
        oracle.use_library(so)

    yield use
    oracle.use_library(None)
    for so in libs:
        shutil.rmtree(os.path.dirname(so), ignore_errors=True)


# --- pins, as functions returning True when the pin passes ---------------------------------

def pin_noise_free_decay():
    p = W.config2()
    c, rho = oracle.meanfield(oracle.OracleProblem(p), 1)
    return np.max(np.abs(rho - A_pow(field_np(p.rho0, p.box, p.n(1)), p.steps(1), p.mu))) < 1e-12


def pin_one_step_law():
    base = W.config2(N=300.0)
    phi = base.obs[0].phi
    p = base.with_(levels=1, T=base.tau(0), obs=[W.Obs(phi, True, True, W.PSI_ID)])
    X = oracle.run_range(oracle.OracleProblem(p), 0, 0, 3000)[:, 0, 0]
    s2 = one_step_sigma2(p, 0, phi)
    return stats.kstest(X / math.sqrt(s2), "norm").pvalue > 1e-4


def pin_pair_variance():
    base = W.config2(N=1e8)
    phi = base.obs[0].phi
    p = base.with_(obs=[W.Obs(phi, True, True, W.PSI_ID)])
    P = oracle.run_range(oracle.OracleProblem(p), 1, 0, 2000)
    Y = P[:, 0, 0] - P[:, 0, 1]
    V = pair_variance_linear(p, 1, phi)
    return abs(Y.var(ddof=1) / V - 1.0) < 4.5 * math.sqrt(2.0 / len(Y))


def pin_restricted_law():
    p = W.config2(N=1e4)
    op = oracle.OracleProblem(p)
    zs = np.stack([oracle.run_pair(op, 1, s, want_coarse_noise=True)[1] for s in range(300)]).reshape(-1)
    return abs(zs.var() - 1.0) < 4.5 * math.sqrt(2.0 / zs.size) and stats.kstest(zs, "norm").pvalue > 1e-4


def pin_dense_divergence():
    from test_oracle_operators import dense_divergence, dense_laplacian, flux_field
    n, h, tau, N = 8, 1 / 8, 0.1 / 64, 37.0
    rng = np.random.default_rng(0)
    rho = 1.0 + 0.8 * rng.standard_normal((n, n))
    db = math.sqrt(tau) * rng.standard_normal((n, n, 2))
    expect = rho.reshape(-1) + 0.5 * tau * dense_laplacian(n, h) @ rho.reshape(-1) + \
        dense_divergence(n, h, 0) @ flux_field(rho, db, h, 0).reshape(-1) / math.sqrt(N)
    return np.max(np.abs(oracle.em_step(rho, db, h, tau, N, 0).reshape(-1) - expect)) < 1e-12


def pin_gauss_vs_fp64():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2 ** 32, size=1 << 16, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2 ** 32, size=1 << 16, dtype=np.uint64).astype(np.uint32)
    z0, z1 = oracle.gauss_pair(a, b)
    u = (2.0 * (a.astype(np.uint64) >> 9).astype(np.float64) + 1.0) * 2.0 ** -24
    th = 2 * math.pi * ((b.astype(np.uint64) >> 30) + (2.0 * ((b.astype(np.uint64) >> 7) & 0x7FFFFF) + 1) * 2.0 ** -24) / 4
    R = np.sqrt(-2 * np.log(u))
    return np.all(np.abs(z0 - R * np.cos(th)) <= 1e-6 * np.maximum(1, R)) and \
        np.all(np.abs(z1 - R * np.sin(th)) <= 1e-6 * np.maximum(1, R))


def pin_bump_fields():
    import test_oracle_fields as F
    try:
        for n in (64, 128):
            for c in ((0.5, 0.5), (0.05, 0.05)):
                F.test_bump_integral_and_second_moment(n, c)
            F.test_bump_peak_on_the_centre_point(n)
    except AssertionError:
        return False
    return True


def pin_clipped_field():
    import test_oracle_fields as F
    try:
        for n in (8, 64):
            F.test_clipped_datum_mean_floor_and_max(n)
    except AssertionError:
        return False
    return True


MUTANTS = [
    # (name, old text, new text, pin that must fail)
    ("coarse increment without 2^{-d/2}", "dbc[k] *= 0.5;   /* 2^{-d/2}, d = 2 */", "dbc[k] *= 1.0;",
     pin_restricted_law),
    ("right-most block shifted by one fine cell",
     "dbc[2 * (a + nc * b) + r] += dbf[2 * ((2 * a + v1) + nf * (2 * b + v2)) + r];",
     "dbc[2 * (a + nc * b) + r] += dbf[2 * (((2 * a + v1 + 1) % nf) + nf * (2 * b + v2)) + r];",
     pin_pair_variance),
    ("coarse step taken with the fine time step", "dko_em_step(nc, hc, tc, p->N, p->flux, rc, dbc, rcn);",
     "dko_em_step(nc, hc, tf, p->N, p->flux, rc, dbc, rcn);", pin_pair_variance),
    ("missing 1/2 in front of the Laplacian", "out[s] = rho[s] + tau * 0.5 * lap + invsqrtN * div;",
     "out[s] = rho[s] + tau * lap + invsqrtN * div;", pin_noise_free_decay),
    ("noise basis without h^{-d/2}", "double hd2 = 1.0 / h;   /* h^{-d/2} with d = 2 */", "double hd2 = 1.0;",
     pin_one_step_law),
    ("divergence with the wrong sign",
     "div = (b[2 * xp + 0] - b[2 * xm + 0]) / (2.0 * h) + (b[2 * yp + 1] - b[2 * ym + 1]) / (2.0 * h);",
     "div = (b[2 * xm + 0] - b[2 * xp + 0]) / (2.0 * h) + (b[2 * yp + 1] - b[2 * ym + 1]) / (2.0 * h);",
     pin_dense_divergence),
    ("absolute value instead of the positive part",
     "double r = rho[s] > 0.0 ? rho[s] : 0.0;", "double r = fabs(rho[s]);", pin_dense_divergence),
    ("Box-Muller quadrant rotated the wrong way", "case 1: c = -sq; sn = cq; break;",
     "case 1: c = sq; sn = -cq; break;", pin_gauss_vs_fp64),
    ("bump width sigma^2 in place of 2 sigma^2",
     "exp(-(dx * dx + dy * dy) / (2.0 * f->bump_sigma * f->bump_sigma))",
     "exp(-(dx * dx + dy * dy) / (f->bump_sigma * f->bump_sigma))", pin_bump_fields),
    ("bump distance without the periodic wrap", "if (d > 0.5 * box) d = box - d;", "", pin_bump_fields),
    ("floor added inside the positive part", "if (f->kind == FIELD_CLIPPED) v = (v > 0.0 ? v : 0.0) + f->floor_add;",
     "if (f->kind == FIELD_CLIPPED) v = (v + f->floor_add > 0.0 ? v + f->floor_add : 0.0);", pin_clipped_field),
]


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_reject_mutant(mutant, name, old, new, pin):
    assert pin(), f"pin {pin.__name__} fails on the regular oracle"
    mutant(old, new)
    assert not pin(), f"mutant '{name}' passes {pin.__name__}"
