"""FP64 CPU oracle for the MLMC Dean--Kawasaki hot path.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package.  It shares no code with the HIP path
(``paper_2311_08872_amd``) and never imports it.  The only common module is
``dk_workloads``, which describes problems and holds none of the method's arithmetic.

Contents
--------
* ``libdk_oracle.so`` (``dk_oracle.c``): Philox4x32-10 (SC'11), the binary32 Box--Muller
  transform, the explicit EM step of eq. (FullyDiscreteDK), single-level and NN-coupled
  (Sec. 3.2) sample paths, observables of eq. (eqn_MLMCLevels) and the discrete mean field.
* ``mlmc.py``: the MLMC estimator of eq. (MLMCEstimator) and Algorithm 1 of Sec. 7
  (optimal sample counts eq. (opt_M_ell), convergence test eq. (convergence_criterion)).
"""
from __future__ import annotations

import ctypes as C
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import dk_workloads as W

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


class _Mode(C.Structure):
    _fields_ = [("amp", C.c_double), ("kx", C.c_double), ("ky", C.c_double), ("phase", C.c_double)]


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_modes", C.c_int32), ("c0", C.c_double),
                ("modes", C.POINTER(_Mode)), ("floor_add", C.c_double),
                ("bump_amp", C.c_double), ("bump_sigma", C.c_double), ("bump_cx", C.c_double),
                ("bump_cy", C.c_double), ("es_a", C.c_double), ("es_b", C.c_double),
                ("es_s", C.c_double), ("es_x0", C.c_double), ("es_y0", C.c_double),
                ("es_scale", C.c_double)]


class _Obs(C.Structure):
    _fields_ = [("phi", _Field), ("centre", C.c_int32), ("scale_sqrtN", C.c_int32),
                ("psi", C.c_int32), ("pad", C.c_int32)]


class _Problem(C.Structure):
    _fields_ = [("box", C.c_double), ("n0", C.c_int32), ("levels", C.c_int32), ("mu", C.c_double),
                ("N", C.c_double), ("steps0", C.c_int32), ("flux", C.c_int32), ("n_obs", C.c_int32),
                ("cell_centred", C.c_int32), ("obs", C.POINTER(_Obs)), ("rho0", _Field), ("seed", C.c_uint64)]


def _load(path):
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    u32p = C.POINTER(C.c_uint32)
    L.dko_philox_many.argtypes = [C.c_int64, u32p, u32p, u32p]
    L.dko_gauss_many.argtypes = [C.c_int64, u32p, u32p, C.POINTER(C.c_float), C.POINTER(C.c_float)]
    L.dko_noise_step.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_uint64, C.c_int, C.c_int, dp]
    L.dko_noise_step_f32.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_uint64, C.c_int, C.c_int,
                                     C.POINTER(C.c_float)]
    L.dko_em_step.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, dp, dp, dp]
    L.dko_field_grid.argtypes = [C.POINTER(_Field), C.c_double, C.c_int, dp]
    L.dko_field_grid_at.argtypes = [C.POINTER(_Field), C.c_double, C.c_int, C.c_double, dp]
    L.dko_meanfield.argtypes = [C.POINTER(_Problem), C.c_int, dp, dp]
    L.dko_run_single.argtypes = [C.POINTER(_Problem), C.c_int, C.c_uint64, C.c_uint32, dp, dp, dp]
    L.dko_run_pair.argtypes = [C.POINTER(_Problem), C.c_int, C.c_uint64, C.c_uint32, dp, dp, dp,
                               dp, dp, dp]
    L.dko_run_range.argtypes = [C.POINTER(_Problem), C.c_int, C.c_int, C.c_uint64, C.c_uint64,
                                C.c_uint32, dp, dp, dp]
    return L


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "libdk_oracle.so")
        if not os.path.exists(path):
            _build.build()
        _lib = _load(path)
    return _lib


def use_library(path: str | None):
    """Swap the oracle library (tests load deliberately broken builds to check that the pins
    reject them); None restores the regular build."""
    global _lib
    _lib = None if path is None else _load(path)


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _field(f: W.Field, keep: list) -> _Field:
    nm = len(f.modes)
    arr = (_Mode * max(nm, 1))()
    for i, m in enumerate(f.modes):
        arr[i] = _Mode(m.amp, m.kx, m.ky, m.phase)
    keep.append(arr)
    return _Field(f.kind, nm, f.c0, C.cast(arr, C.POINTER(_Mode)), f.floor_add, f.bump_amp,
                  f.bump_sigma, f.bump_cx, f.bump_cy, f.es_a, f.es_b, f.es_s, f.es_x0, f.es_y0,
                  f.es_scale)


class OracleProblem:
    """Marshalled copy of a ``dk_workloads.Problem`` for the oracle library."""

    def __init__(self, p: W.Problem):
        self.p = p
        self._keep = []
        obs = (_Obs * max(len(p.obs), 1))()
        for i, o in enumerate(p.obs):
            obs[i] = _Obs(_field(o.phi, self._keep), int(o.centre), int(o.scale_sqrtN), int(o.psi), 0)
        self._keep.append(obs)
        assert p.coupling == W.COUPLING_NN, "the library oracle runs the NN coupling; see oracle.fourier"
        self.c = _Problem(p.box, p.n0, p.levels, p.mu, p.N, p.steps(0), p.flux, len(p.obs), int(p.grid == W.GRID_CELL),
                          C.cast(obs, C.POINTER(_Obs)), _field(p.rho0, self._keep), p.seed)
        self._centres = {}

    @property
    def ref(self):
        return C.byref(self.c)

    def centre(self, level: int) -> np.ndarray:
        """Centring constants c_{l,j} = (rho_bar_l^M, I_h phi_j)_h (FP64 noise-free run)."""
        if level not in self._centres:
            c = np.zeros(max(len(self.p.obs), 1))
            lib().dko_meanfield(self.ref, level, _dp(c), None)
            self._centres[level] = c
        return self._centres[level]


# ------------------------------------------------------------------------------------------
# Generator
# ------------------------------------------------------------------------------------------

def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros_like(ctr)
    u32p = C.POINTER(C.c_uint32)
    lib().dko_philox_many(len(ctr), ctr.ctypes.data_as(u32p), key.ctypes.data_as(u32p),
                          out.ctypes.data_as(u32p))
    return out


def gauss_pair(a: np.ndarray, b: np.ndarray):
    a = np.ascontiguousarray(a, dtype=np.uint32).ravel()
    b = np.ascontiguousarray(b, dtype=np.uint32).ravel()
    z0 = np.zeros(len(a), np.float32)
    z1 = np.zeros(len(a), np.float32)
    u32p = C.POINTER(C.c_uint32)
    fp = C.POINTER(C.c_float)
    lib().dko_gauss_many(len(a), a.ctypes.data_as(u32p), b.ctypes.data_as(u32p),
                         z0.ctypes.data_as(fp), z1.ctypes.data_as(fp))
    return z0, z1


def noise_step(seed: int, tag: int, level: int, sample: int, n: int, m: int, f32: bool = False):
    """Standard normals of one fine step, shape (n, n, 2) indexed [y, x, r]."""
    if f32:
        z = np.zeros(2 * n * n, np.float32)
        lib().dko_noise_step_f32(seed, tag, level, sample, n, m, z.ctypes.data_as(C.POINTER(C.c_float)))
    else:
        z = np.zeros(2 * n * n)
        lib().dko_noise_step(seed, tag, level, sample, n, m, _dp(z))
    return z.reshape(n, n, 2)


# ------------------------------------------------------------------------------------------
# Scheme
# ------------------------------------------------------------------------------------------

def em_step(rho: np.ndarray, dbeta: np.ndarray, h: float, tau: float, N: float, flux: int = 0):
    """One explicit EM step; rho [y, x], dbeta [y, x, r] (already scaled by sqrt(tau))."""
    n = rho.shape[0]
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    dbeta = np.ascontiguousarray(dbeta, dtype=np.float64)
    out = np.zeros_like(rho)
    lib().dko_em_step(n, h, tau, N, flux, _dp(rho), _dp(dbeta), _dp(out))
    return out


def field_grid(f: W.Field, box: float, n: int, offset: float = 0.0) -> np.ndarray:
    """I_h f at the points ((i + offset) h, (j + offset) h), shape [y, x]."""
    keep = []
    cf = _field(f, keep)
    out = np.zeros(n * n)
    lib().dko_field_grid_at(C.byref(cf), box, n, offset, _dp(out))
    return out.reshape(n, n)


def meanfield(op: OracleProblem, level: int):
    n = op.p.n(level)
    c = np.zeros(max(len(op.p.obs), 1))
    rho = np.zeros(n * n)
    lib().dko_meanfield(op.ref, level, _dp(c), _dp(rho))
    return c, rho.reshape(n, n)


def run_single(op: OracleProblem, level: int, sample: int, tag: int = W.TAG_MLMC, want_field=False):
    n = op.p.n(level)
    P = np.zeros(max(len(op.p.obs), 1))
    rho = np.zeros(n * n) if want_field else None
    lib().dko_run_single(op.ref, level, sample, tag, _dp(op.centre(level)), _dp(P), _dp(rho))
    return (P, rho.reshape(n, n)) if want_field else P


def run_pair(op: OracleProblem, level: int, sample: int, tag: int = W.TAG_MLMC, want_field=False,
             want_coarse_noise=False):
    nf = op.p.n(level)
    nc = nf // 2
    P = np.zeros(2 * max(len(op.p.obs), 1))
    rf = np.zeros(nf * nf) if want_field else None
    rc = np.zeros(nc * nc) if want_field else None
    zc = np.zeros(2 * nc * nc) if want_coarse_noise else None
    lib().dko_run_pair(op.ref, level, sample, tag, _dp(op.centre(level)), _dp(op.centre(level - 1)),
                       _dp(P), _dp(rf), _dp(rc), _dp(zc))
    out = [P.reshape(-1, 2)]
    if want_field:
        out += [rf.reshape(nf, nf), rc.reshape(nc, nc)]
    if want_coarse_noise:
        out += [zc.reshape(nc, nc, 2)]
    return out[0] if len(out) == 1 else tuple(out)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def run_range(op: OracleProblem, level: int, first: int, count: int, tag: int = W.TAG_MLMC,
              coupled: bool | None = None, threads: int | None = None) -> np.ndarray:
    """Per-sample (P_fine, P_coarse) for samples [first, first+count): shape (count, n_obs, 2).

    ``coupled`` defaults to ``level >= 1`` (a level pair); for level 0 or plain MC the
    coarse column is zero."""
    if coupled is None:
        coupled = level >= 1
    nobs = max(len(op.p.obs), 1)
    out = np.zeros((count, nobs, 2))
    cf = op.centre(level)
    cc = op.centre(level - 1) if coupled else cf
    threads = threads or default_threads()
    chunks = []
    step = max(1, (count + threads - 1) // threads)
    for s in range(0, count, step):
        chunks.append((s, min(count, s + step)))

    def work(ch):
        s, e = ch
        buf = np.zeros((e - s, nobs, 2))
        lib().dko_run_range(op.ref, level, int(coupled), first + s, e - s, tag, _dp(cf), _dp(cc), _dp(buf))
        out[s:e] = buf

    if len(chunks) == 1:
        work(chunks[0])
    else:
        with ThreadPoolExecutor(len(chunks)) as ex:
            list(ex.map(work, chunks))
    return out
