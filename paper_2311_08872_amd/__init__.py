"""MI355X (gfx950) MLMC for the Dean--Kawasaki equation: Python binding of libdk_mlmc.so.

Every computation runs in the HIP library; this module only marshals arguments.  PyTorch is
used for device buffers and streams.  The function names follow the C ABI
(include/dk_mlmc.h): ``level_pair`` (dk_mlmc_level_pair), ``mc_level`` (dk_mc_level),
``estimate`` (dk_mlmc_estimate), ``meanfield`` (dk_meanfield), ``noise_dump``
(dk_noise_dump), ``level_fields`` (dk_level_fields) and ``alg1_host`` (dk_alg1_host).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np

import dk_workloads as W

from . import _lib as L

__all__ = ["Context", "Moments", "level_pair", "mc_level", "estimate", "meanfield", "noise_dump",
           "level_fields", "alg1_host", "cnn_init", "cnn_forward", "cnn_loss_grad", "cv_train", "DKError"]


class DKError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dk error {code}: {msg}")
        self.code = code


def _check(rc: int) -> int:
    if rc < 0:
        raise DKError(rc, L.load().dk_last_error().decode(errors="replace"))
    return rc


# ------------------------------------------------------------------------------------------
# Problem marshalling
# ------------------------------------------------------------------------------------------

def _field(f: W.Field, keep: list) -> L.dk_field:
    n = len(f.modes)
    arr = (L.dk_mode * max(n, 1))()
    for i, m in enumerate(f.modes):
        arr[i] = L.dk_mode(m.amp, m.kx, m.ky, m.phase)
    keep.append(arr)
    return L.dk_field(f.kind, n, f.c0, C.cast(arr, C.POINTER(L.dk_mode)), f.floor_add, f.bump_amp, f.bump_sigma,
                      f.bump_cx, f.bump_cy, f.es_a, f.es_b, f.es_s, f.es_x0, f.es_y0, f.es_scale)


class CProblem:
    """A dk_problem struct (and the arrays it points to) built from a dk_workloads.Problem."""

    def __init__(self, p: W.Problem):
        self.p = p
        self._keep = []
        obs = (L.dk_obs * max(len(p.obs), 1))()
        for i, o in enumerate(p.obs):
            obs[i] = L.dk_obs(_field(o.phi, self._keep), int(o.centre), int(o.scale_sqrtN), int(o.psi), 0)
        self._keep.append(obs)
        self.c = L.dk_problem(2, p.n0, p.levels, p.steps_policy, p.box, p.mu, p.T, p.N, p.flux, p.precision,
                              len(p.obs), p.primary, C.cast(obs, C.POINTER(L.dk_obs)), _field(p.rho0, self._keep),
                              p.seed, p.coupling, p.grid, float(p.b0))

    @property
    def ref(self):
        return C.byref(self.c)


def _cp(problem) -> CProblem:
    return problem if isinstance(problem, CProblem) else CProblem(problem)


@dataclass
class Moments:
    count: int
    sums: np.ndarray   # [DK_NMOM]: Y, Y^2, Pf, Pf^2, Pc, Pc^2 (compensated values)

    def stats(self, q: int = 0):
        """(mean, unbiased variance) of Y (q = 0), P_fine (1) or P_coarse (2): dk_moments_mean_var."""
        m = L.dk_moments()
        m.count = self.count
        for k in range(L.DK_NMOM):
            m.sum[k] = float(self.sums[k])
            m.comp[k] = 0.0
        mean, var = C.c_double(), C.c_double()
        _check(L.load().dk_moments_mean_var(C.byref(m), q, C.byref(mean), C.byref(var)))
        return mean.value, var.value

    @property
    def mean(self) -> float:
        return self.stats(0)[0]

    @property
    def var(self) -> float:
        return self.stats(0)[1]


def _moments(arr) -> List[Moments]:
    out = []
    for m in arr:
        out.append(Moments(int(m.count), np.array([m.sum[k] + m.comp[k] for k in range(L.DK_NMOM)])))
    return out


# ------------------------------------------------------------------------------------------
# Context and streams
# ------------------------------------------------------------------------------------------

def _torch():
    import torch
    return torch


class Context:
    def __init__(self, device: int = 0):
        self.lib = L.load()
        self.device = device
        h = C.c_void_p()
        _check(self.lib.dk_context_create(C.byref(h), device))
        self.h = h

    def close(self):
        if self.h:
            self.lib.dk_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> list:
        """Per (level, coupled) kernel timings recorded with HIP events since the last reset."""
        n = _check(self.lib.dk_context_stats(self.h, None, 0))
        arr = (L.dk_kernel_stats * max(n, 1))()
        n = _check(self.lib.dk_context_stats(self.h, arr, n))
        return [{"level": r.level, "coupled": bool(r.coupled), "launches": r.launches, "samples": r.samples,
                 "kernel_ms": r.kernel_ms, "cell_updates": r.cell_updates, "rows": r.rows} for r in arr[:n]]

    def set_shape(self, n: int, variant: int):
        """Force tile-shape variant `variant` for grid size n (-1: automatic)."""
        _check(self.lib.dk_context_set_shape(self.h, n, variant))

    def tuning_json(self) -> str:
        """The autotuner's tile-shape and streaming-depth choices as JSON text."""
        n = _check(self.lib.dk_context_tuning_json(self.h, None, 0))
        buf = C.create_string_buffer(n + 1)
        _check(self.lib.dk_context_tuning_json(self.h, buf, n + 1))
        return buf.value.decode()

    def load_tuning_json(self, text: str):
        """Use tile-shape choices from JSON text (as written by tuning_json) without timing."""
        _check(self.lib.dk_context_load_tuning_json(self.h, text.encode()))

    def set_launch_cap(self, cells: float):
        """Largest work of one sampling launch in cell updates (0 = default 2e12)."""
        _check(self.lib.dk_context_set_launch_cap(self.h, float(cells)))

    def set_streaming(self, on: bool):
        """Route levels of size >= 64 through the HBM-streaming kernel (comparison / testing)."""
        _check(self.lib.dk_context_set_streaming(self.h, int(on)))

    def set_stream_depth(self, depth: int):
        """Temporal depth of the streaming kernel: 1, 2, 4 or 8 fine steps per launch (0: automatic)."""
        _check(self.lib.dk_context_set_stream_depth(self.h, int(depth)))

    @staticmethod
    def shape_rows(n: int, variant: int) -> int:
        return L.load().dk_shape_rows(n, variant)

    @staticmethod
    def shape_spw(n: int, variant: int) -> int:
        return L.load().dk_shape_spw(n, variant)

    def reset(self, drop_tables: bool = False):
        _check(self.lib.dk_context_reset(self.h, int(drop_tables)))

    def stream(self):
        torch = _torch()
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)


_default_ctx: Optional[Context] = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context(0)
    return _default_ctx


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


# ------------------------------------------------------------------------------------------
# Entry points
# ------------------------------------------------------------------------------------------

def level_pair(problem, level: int, first: int, n: int, tag: int = W.TAG_MLMC, per_sample: bool = False,
               ctx: Context | None = None):
    """dk_mlmc_level_pair: moments per observable, and optionally the per-sample (P_f, P_c)
    as a float64 device tensor of shape (n, n_obs, 2)."""
    ctx = ctx or default_context()
    cp = _cp(problem)
    nobs = len(cp.p.obs)
    sums = (L.dk_moments * nobs)()
    out = None
    if per_sample:
        torch = _torch()
        out = torch.empty((n, nobs, 2), dtype=torch.float64, device=f"cuda:{ctx.device}")
    _check(ctx.lib.dk_mlmc_level_pair(ctx.h, cp.ref, level, first, n, tag, sums, _ptr(out), ctx.stream()))
    return (_moments(sums), out) if per_sample else _moments(sums)


def level_pair_noalloc(problem, level: int, first: int, n: int, tag: int = W.TAG_MLMC, per_sample: bool = False,
                       device: int = 0, stream=None):
    """dk_mlmc_level_pair_noalloc: as level_pair, on the current device, with the library's fixed
    device workspace (no context, no device allocation inside the call).  The optional per-sample
    output tensor is allocated here, by the caller's side of the boundary."""
    lib = L.load()
    cp = _cp(problem)
    nobs = len(cp.p.obs)
    sums = (L.dk_moments * nobs)()
    out = None
    torch = _torch()
    if per_sample:
        out = torch.empty((n, nobs, 2), dtype=torch.float64, device=f"cuda:{device}")
    if stream is None:
        stream = torch.cuda.current_stream(device).cuda_stream
    with torch.cuda.device(device):
        _check(lib.dk_mlmc_level_pair_noalloc(cp.ref, level, first, n, tag, sums, _ptr(out), C.c_void_p(stream)))
    return (_moments(sums), out) if per_sample else _moments(sums)


def mc_level(problem, level: int, first: int, n: int, per_sample: bool = False, ctx: Context | None = None):
    ctx = ctx or default_context()
    cp = _cp(problem)
    nobs = len(cp.p.obs)
    sums = (L.dk_moments * nobs)()
    out = None
    if per_sample:
        torch = _torch()
        out = torch.empty((n, nobs, 2), dtype=torch.float64, device=f"cuda:{ctx.device}")
    _check(ctx.lib.dk_mc_level(ctx.h, cp.ref, level, first, n, sums, _ptr(out), ctx.stream()))
    return (_moments(sums), out) if per_sample else _moments(sums)


def round_sums(problem, finest: int, first, count, tag: int = W.TAG_MLMC, round_mode: int = 0,
               ctx: Context | None = None):
    """dk_mlmc_round: one Algorithm-1 round of samples [first[l], first[l] + count[l]) of levels
    0..finest in the given round mode; returns moments [finest + 1][n_obs]."""
    ctx = ctx or default_context()
    cp = _cp(problem)
    nobs = len(cp.p.obs)
    f = (C.c_uint64 * (finest + 1))(*[int(v) for v in first])
    c = (C.c_uint64 * (finest + 1))(*[int(v) for v in count])
    sums = (L.dk_moments * ((finest + 1) * nobs))()
    _check(ctx.lib.dk_mlmc_round(ctx.h, cp.ref, finest, f, c, tag, round_mode, sums, ctx.stream()))
    ms = _moments(sums)
    return [ms[l * nobs:(l + 1) * nobs] for l in range(finest + 1)]


def _opts(m_pilot=1000, L_start=2, alpha=2.0, max_rounds=1000, plain_mc_level=-1, max_samples=0, cv_params=None,
          cv_level_mask=0, cv_ratio=4, round_mode=0, checkpoint_path=None, cost_model=0, _keep=None):
    ptr = None
    if cv_params is not None:
        arr = np.ascontiguousarray(cv_params, dtype=np.float32)
        if _keep is not None:
            _keep.append(arr)
        ptr = arr.ctypes.data_as(C.POINTER(C.c_float))
    ck = None
    if checkpoint_path is not None:
        ck = str(checkpoint_path).encode()
        if _keep is not None:
            _keep.append(ck)
    return L.dk_mlmc_opts(m_pilot, L_start, alpha, max_rounds, plain_mc_level, max_samples, ptr, cv_level_mask,
                          cv_ratio, round_mode, cost_model, ck)


def _result_dict(r: L.dk_mlmc_result, nobs: int, rc: int) -> dict:
    Lv = r.L
    return {"status": rc, "estimate": list(r.estimate[:nobs]), "var_est": list(r.var_est[:nobs]),
            "bias_est": r.bias_est, "rmse_est": r.rmse_est, "L": Lv, "converged": bool(r.converged),
            "rounds": r.rounds, "M": list(r.M[:Lv + 1]), "Yhat": list(r.Yhat[:Lv + 1]),
            "Vhat": list(r.Vhat[:Lv + 1]), "cost": list(r.cost[:Lv + 1]), "cell_updates": r.cell_updates,
            "wall_s": r.wall_s}


def estimate(problem, eps: float, ctx: Context | None = None, level_moments: bool = False, **opts) -> dict:
    """dk_mlmc_estimate: Algorithm 1 to RMSE eps (or plain MC with plain_mc_level=l)."""
    ctx = ctx or default_context()
    cp = _cp(problem)
    nobs = len(cp.p.obs)
    keep = []
    o = _opts(_keep=keep, **opts)
    r = L.dk_mlmc_result()
    mom = (L.dk_moments * (cp.p.levels * nobs))() if level_moments else None
    rc = _check(ctx.lib.dk_mlmc_estimate(ctx.h, cp.ref, eps, C.byref(o), C.byref(r), mom, ctx.stream()))
    d = _result_dict(r, nobs, rc)
    if level_moments:
        ms = _moments(mom)
        d["level_moments"] = [ms[l * nobs:(l + 1) * nobs] for l in range(cp.p.levels)]
    return d


def meanfield(problem, level: int, want_field: bool = False, ctx: Context | None = None):
    ctx = ctx or default_context()
    cp = _cp(problem)
    nobs = len(cp.p.obs)
    c = (C.c_double * nobs)()
    rho = None
    if want_field:
        torch = _torch()
        n = cp.p.n(level)
        rho = torch.empty((n, n), dtype=torch.float64, device=f"cuda:{ctx.device}")
    _check(ctx.lib.dk_meanfield(ctx.h, cp.ref, level, c, _ptr(rho), ctx.stream()))
    cen = np.array(c[:])
    return (cen, rho) if want_field else cen


def noise_dump(seed: int, tag: int, level: int, n: int, first_sample: int, n_samples: int, first_step: int,
               n_steps: int, ctx: Context | None = None):
    """dk_noise_dump: float32 device tensor [n_samples, n_steps, n, n, 2] ([..., y, x, r])."""
    ctx = ctx or default_context()
    torch = _torch()
    out = torch.empty((n_samples, n_steps, n, n, 2), dtype=torch.float32, device=f"cuda:{ctx.device}")
    _check(ctx.lib.dk_noise_dump(ctx.h, seed, tag, level, n, first_sample, n_samples, first_step, n_steps,
                                 _ptr(out), ctx.stream()))
    return out


def gauss_transform(a, b, ctx: Context | None = None):
    """dk_gauss_transform: the generator's two normals of each word pair (a[i], b[i]).  a, b:
    int32 device tensors holding the uint32 words (same length); returns float32 (z0, z1)."""
    ctx = ctx or default_context()
    torch = _torch()
    if a.dtype != torch.int32 or b.dtype != torch.int32 or a.shape != b.shape or not a.is_cuda or not b.is_cuda:
        raise DKError(-1, "a and b must be int32 CUDA tensors of one shape")
    a = a.contiguous()
    b = b.contiguous()
    z0 = torch.empty(a.shape, dtype=torch.float32, device=a.device)
    z1 = torch.empty(a.shape, dtype=torch.float32, device=a.device)
    _check(ctx.lib.dk_gauss_transform(ctx.h, _ptr(a), _ptr(b), a.numel(), _ptr(z0), _ptr(z1), ctx.stream()))
    return z0, z1


def level_fields(problem, level: int, coupled: bool, first: int, n: int, tag: int = W.TAG_MLMC,
                 ctx: Context | None = None):
    """dk_level_fields: (per-sample (n, n_obs, 2), rho_f (n, nf, nf), rho_c (n, nc, nc) or None)."""
    ctx = ctx or default_context()
    torch = _torch()
    cp = _cp(problem)
    nobs = len(cp.p.obs)
    dt = torch.float64 if cp.p.precision == W.PREC_F64 else torch.float32
    nf = cp.p.n(level)
    dev = f"cuda:{ctx.device}"
    ps = torch.empty((n, nobs, 2), dtype=torch.float64, device=dev)
    rf = torch.empty((n, nf, nf), dtype=dt, device=dev)
    rc = torch.empty((n, nf // 2, nf // 2), dtype=dt, device=dev) if coupled else None
    _check(ctx.lib.dk_level_fields(ctx.h, cp.ref, level, int(coupled), first, n, tag, _ptr(ps), _ptr(rf), _ptr(rc),
                                   ctx.stream()))
    return ps, rf, rc


def cnn_init(seed: int = 0) -> np.ndarray:
    """dk_cnn_init: seeded He initialisation of the network parameters (float32 [5953])."""
    lib = L.load()
    out = np.zeros(L.DK_CNN_NPARAM, np.float32)
    _check(lib.dk_cnn_init(seed, out.ctypes.data_as(C.POINTER(C.c_float))))
    return out


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def cnn_forward(params: np.ndarray, x, ctx: Context | None = None):
    """dk_cnn_forward: x float32 device tensor [batch, n, n] -> float32 device tensor [batch]."""
    ctx = ctx or default_context()
    torch = _torch()
    params = np.ascontiguousarray(params, dtype=np.float32)
    x = x.contiguous()
    r = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    _check(ctx.lib.dk_cnn_forward(ctx.h, _fptr(params), x.shape[1], x.shape[0], _ptr(x), _ptr(r), ctx.stream()))
    return r


def cnn_loss_grad(params: np.ndarray, x, y, ctx: Context | None = None):
    """dk_cnn_loss_grad: (mean squared error, gradient float32 [5953]) on device tensors x, y."""
    ctx = ctx or default_context()
    params = np.ascontiguousarray(params, dtype=np.float32)
    x = x.contiguous()
    y = y.contiguous()
    g = np.zeros(L.DK_CNN_NPARAM, np.float32)
    loss = C.c_double()
    _check(ctx.lib.dk_cnn_loss_grad(ctx.h, _fptr(params), x.shape[1], x.shape[0], _ptr(x), _ptr(y), _fptr(g),
                                    C.byref(loss), ctx.stream()))
    return loss.value, g


def cv_train(problem, level: int, n_train: int = 1 << 16, epochs: int = 10, batch: int = 256, lr: float = 1e-3,
             n_val: int = 8192, params: np.ndarray | None = None, seed: int = 0, ctx: Context | None = None) -> dict:
    """dk_cv_train: train the control-variate network of `level` on the GPU."""
    ctx = ctx or default_context()
    cp = _cp(problem)
    prm = np.ascontiguousarray(cnn_init(seed) if params is None else params, dtype=np.float32).copy()
    hist = np.zeros(epochs)
    val = np.zeros(3)
    _check(ctx.lib.dk_cv_train(ctx.h, cp.ref, level, n_train, epochs, batch, lr, n_val, _fptr(prm),
                               hist.ctypes.data_as(C.POINTER(C.c_double)), val.ctypes.data_as(C.POINTER(C.c_double)),
                               ctx.stream()))
    return {"params": prm, "loss": hist.tolist(), "var_Y": val[0], "var_Y_minus_r": val[1], "var_r": val[2]}


def heat_steps(rho, steps: int, mu: float, ctx: Context | None = None) -> float:
    """dk_heat_steps: noise-free steps of a batch of FP32 fields rho [batch, n, n] (device,
    in place); returns the kernel time in ms."""
    ctx = ctx or default_context()
    torch = _torch()
    assert rho.dtype == torch.float32 and rho.is_contiguous()
    work = torch.empty_like(rho)
    ms = C.c_double()
    _check(ctx.lib.dk_heat_steps(ctx.h, rho.shape[-1], rho.shape[0], steps, mu, _ptr(rho), _ptr(work), C.byref(ms),
                                 ctx.stream()))
    return ms.value


def alg1_host(eps: float, L_max: int, cost, sampler: Callable[[int, int, int], np.ndarray], **opts) -> dict:
    """dk_alg1_host: the library's Algorithm 1 over a Python level sampler (no GPU).
    sampler(level, first, count) returns the values Y of those samples."""
    lib = L.load()
    err = []

    def cb(user, level, first, count, sums):
        try:
            y = np.asarray(sampler(int(level), int(first), int(count)), dtype=np.float64)
            sums[0] = float(np.sum(y))
            sums[1] = float(np.sum(y * y))
            return 0
        except Exception as e:   # reported as an error code through the ABI
            err.append(e)
            return -1

    cfun = L.SAMPLER(cb)
    carr = (C.c_double * (L_max + 1))(*[float(c) for c in cost])
    o = _opts(**opts)
    r = L.dk_mlmc_result()
    rc = lib.dk_alg1_host(eps, L_max, carr, C.byref(o), cfun, None, C.byref(r))
    if err:
        raise err[0]
    _check(rc)
    return _result_dict(r, 1, rc)
