"""Pins for the oracle's random-number generator.

* Philox4x32-10 against rocRAND's own philox4x32_10 engine (an independent implementation
  of the SC'11 definition), run on the CPU through its header-only source.
* The binary32 Box--Muller transform against the FP64 formula z = sqrt(-2 ln u) (cos, sin)(2 pi v)
  evaluated with libm on the exact uniforms, and against the N(0,1) law.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_tool():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    d = tempfile.mkdtemp(prefix="dk_rocrand_")
    exe = os.path.join(d, "rocrand_philox_ref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "native", "rocrand_philox_ref.cpp")],
                          cwd=d)
    yield exe, d
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_tool):
    exe, d = rocrand_tool
    rng = np.random.default_rng(1234)
    rows = rng.integers(0, 2 ** 32, size=(4096, 6), dtype=np.uint64).astype(np.uint32)
    rows[:, 1] &= 0x3FFFFFFF          # keeps 4 (c0 + 2^32 c1) inside 64 bits
    rows[:8] = 0                      # all-zero counter and key
    rows[8:16, 4:] = 0xFFFFFFFF       # all-ones key
    # counters shaped like the ones the scheme uses (site, step, sample, tag|level|sample_hi)
    rows[16:32, 0] = np.arange(16)
    rows[16:32, 1] = 7
    rows[16:32, 2] = 123456
    rows[16:32, 3] = (1 << 24) | (3 << 16)
    fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
    rows.tofile(fin)
    subprocess.check_call([exe, fin, fout])
    ref = np.fromfile(fout, dtype=np.uint32).reshape(-1, 4)
    mine = oracle.philox(rows[:, :4], rows[:, 4:])
    assert np.array_equal(ref, mine)


def _exact_uniforms(a, b):
    a = a.astype(np.uint64)
    b = b.astype(np.uint64)
    u = (2.0 * (a >> 9).astype(np.float64) + 1.0) * 2.0 ** -24
    q = (b >> 30).astype(np.float64)
    f = (2.0 * ((b >> 7) & 0x7FFFFF).astype(np.float64) + 1.0) * 2.0 ** -24
    theta = 2.0 * math.pi * (q + f) / 4.0
    return u, theta


def test_gauss_transform_matches_fp64_box_muller():
    rng = np.random.default_rng(7)
    a = rng.integers(0, 2 ** 32, size=1 << 20, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2 ** 32, size=1 << 20, dtype=np.uint64).astype(np.uint32)
    # extreme radius words and quadrant / octant boundaries of the angle word
    a[:6] = [0, 1, 0x1FF, 0x200, 0xFFFFFFFF, 0x80000000]
    b[:6] = [0, 0x3FFFFFFF, 0x40000000, 0x7FFFFFFF, 0xFFFFFFFF, 0x20000000]
    z0, z1 = oracle.gauss_pair(a, b)
    u, th = _exact_uniforms(a, b)
    R = np.sqrt(-2.0 * np.log(u))
    r0, r1 = R * np.cos(th), R * np.sin(th)
    tol = 1e-6 * np.maximum(1.0, R)
    assert np.all(np.abs(z0 - r0) <= tol), np.max(np.abs(z0 - r0) / tol)
    assert np.all(np.abs(z1 - r1) <= tol), np.max(np.abs(z1 - r1) / tol)
    # the radius is bounded by sqrt(-2 ln 2^-24) (documented tail truncation)
    assert np.max(np.hypot(z0, z1)) <= math.sqrt(48 * math.log(2)) * (1 + 1e-6)


def test_gauss_transform_law():
    rng = np.random.default_rng(11)
    ctr = rng.integers(0, 2 ** 32, size=(1 << 18, 4), dtype=np.uint64).astype(np.uint32)
    key = np.tile(np.array([5, 0], np.uint32), (len(ctr), 1))
    w = oracle.philox(ctr, key)
    z = np.concatenate(oracle.gauss_pair(w[:, 0], w[:, 1]) + oracle.gauss_pair(w[:, 2], w[:, 3])).astype(np.float64)
    n = len(z)
    assert abs(z.mean()) < 4.5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 4.5 * math.sqrt(2.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 4.5 * math.sqrt(96.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the two outputs of one pair are uncorrelated
    z0, z1 = oracle.gauss_pair(w[:, 0], w[:, 1])
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 4.5 / math.sqrt(len(z0))


def test_noise_step_law_and_stream_separation():
    n = 16
    zs = np.stack([oracle.noise_step(0, 0, 2, s, n, m) for s in range(8) for m in range(8)])
    flat = zs.reshape(-1)
    assert abs(flat.mean()) < 4.5 / math.sqrt(flat.size)
    assert abs(flat.var() - 1.0) < 4.5 * math.sqrt(2.0 / flat.size)
    # every (sample, step, tag, level) addresses its own stream
    base = oracle.noise_step(0, 0, 2, 3, n, 5)
    for other in [oracle.noise_step(0, 1, 2, 3, n, 5), oracle.noise_step(0, 0, 1, 3, n, 5),
                  oracle.noise_step(0, 0, 2, 4, n, 5), oracle.noise_step(0, 0, 2, 3, n, 6),
                  oracle.noise_step(1, 0, 2, 3, n, 5), oracle.noise_step(0, 0, 2, 3 + (1 << 32), n, 5)]:
        assert not np.any(base == other)
    # the FP32 and FP64 views of the generator are the same numbers
    assert np.array_equal(oracle.noise_step(0, 0, 2, 3, n, 5, f32=True).astype(np.float64), base)
