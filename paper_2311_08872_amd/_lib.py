"""ctypes declarations of the C ABI in include/dk_mlmc.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdk_mlmc.so")

DK_MAX_OBS = 64
DK_MAX_LEVELS = 12
DK_NMOM = 6
DK_CNN_NPARAM = 5953


class dk_mode(C.Structure):
    _fields_ = [("amp", C.c_double), ("kx", C.c_double), ("ky", C.c_double), ("phase", C.c_double)]


class dk_field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_modes", C.c_int32), ("c0", C.c_double),
                ("modes", C.POINTER(dk_mode)), ("floor_add", C.c_double),
                ("bump_amp", C.c_double), ("bump_sigma", C.c_double), ("bump_cx", C.c_double),
                ("bump_cy", C.c_double), ("es_a", C.c_double), ("es_b", C.c_double), ("es_s", C.c_double),
                ("es_x0", C.c_double), ("es_y0", C.c_double), ("es_scale", C.c_double)]


class dk_obs(C.Structure):
    _fields_ = [("phi", dk_field), ("centre", C.c_int32), ("scale_sqrtN", C.c_int32), ("psi", C.c_int32),
                ("reserved", C.c_int32)]


class dk_problem(C.Structure):
    _fields_ = [("d", C.c_int32), ("n0", C.c_int32), ("levels", C.c_int32), ("steps_policy", C.c_int32),
                ("box", C.c_double), ("mu", C.c_double), ("T", C.c_double), ("N", C.c_double),
                ("flux", C.c_int32), ("precision", C.c_int32), ("n_obs", C.c_int32), ("primary_obs", C.c_int32),
                ("obs", C.POINTER(dk_obs)), ("rho0", dk_field), ("seed", C.c_uint64),
                ("coupling", C.c_int32), ("grid", C.c_int32), ("b0", C.c_double)]


class dk_moments(C.Structure):
    _fields_ = [("count", C.c_uint64), ("sum", C.c_double * DK_NMOM), ("comp", C.c_double * DK_NMOM)]


class dk_mlmc_opts(C.Structure):
    _fields_ = [("m_pilot", C.c_int32), ("L_start", C.c_int32), ("alpha", C.c_double), ("max_rounds", C.c_int32),
                ("plain_mc_level", C.c_int32), ("max_samples", C.c_uint64), ("cv_params", C.POINTER(C.c_float)),
                ("cv_level_mask", C.c_uint32), ("cv_ratio", C.c_int32), ("round_mode", C.c_int32),
                ("cost_model", C.c_int32), ("checkpoint_path", C.c_char_p)]


class dk_mlmc_result(C.Structure):
    _fields_ = [("estimate", C.c_double * DK_MAX_OBS), ("var_est", C.c_double * DK_MAX_OBS),
                ("bias_est", C.c_double), ("rmse_est", C.c_double), ("L", C.c_int32), ("converged", C.c_int32),
                ("rounds", C.c_int32), ("reserved", C.c_int32), ("M", C.c_uint64 * DK_MAX_LEVELS),
                ("Yhat", C.c_double * DK_MAX_LEVELS), ("Vhat", C.c_double * DK_MAX_LEVELS),
                ("cost", C.c_double * DK_MAX_LEVELS), ("cell_updates", C.c_double), ("wall_s", C.c_double)]


class dk_kernel_stats(C.Structure):
    _fields_ = [("level", C.c_int32), ("coupled", C.c_int32), ("launches", C.c_uint64), ("samples", C.c_uint64),
                ("kernel_ms", C.c_double), ("cell_updates", C.c_double), ("rows", C.c_int32), ("reserved", C.c_int32)]


SAMPLER = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int32, C.c_uint64, C.c_uint64, C.POINTER(C.c_double))

# Every symbol include/dk_mlmc.h declares, with (restype, argtypes).
SIGNATURES = {
    "dk_context_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "dk_context_destroy": (None, [C.c_void_p]),
    "dk_mlmc_level_pair": (C.c_int, [C.c_void_p, C.POINTER(dk_problem), C.c_int32, C.c_uint64, C.c_uint64,
                                     C.c_uint32, C.POINTER(dk_moments), C.c_void_p, C.c_void_p]),
    "dk_moments_mean_var": (C.c_int, [C.POINTER(dk_moments), C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "dk_mlmc_level_pair_noalloc": (C.c_int, [C.POINTER(dk_problem), C.c_int32, C.c_uint64, C.c_uint64, C.c_uint32,
                                             C.POINTER(dk_moments), C.c_void_p, C.c_void_p]),
    "dk_mc_level": (C.c_int, [C.c_void_p, C.POINTER(dk_problem), C.c_int32, C.c_uint64, C.c_uint64,
                              C.POINTER(dk_moments), C.c_void_p, C.c_void_p]),
    "dk_mlmc_round": (C.c_int, [C.c_void_p, C.POINTER(dk_problem), C.c_int32, C.POINTER(C.c_uint64),
                                C.POINTER(C.c_uint64), C.c_uint32, C.c_int32, C.POINTER(dk_moments), C.c_void_p]),
    "dk_mlmc_estimate": (C.c_int, [C.c_void_p, C.POINTER(dk_problem), C.c_double, C.POINTER(dk_mlmc_opts),
                                   C.POINTER(dk_mlmc_result), C.POINTER(dk_moments), C.c_void_p]),
    "dk_meanfield": (C.c_int, [C.c_void_p, C.POINTER(dk_problem), C.c_int32, C.POINTER(C.c_double), C.c_void_p,
                               C.c_void_p]),
    "dk_gauss_transform": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "dk_noise_dump": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.c_int32, C.c_int32, C.c_uint64, C.c_uint32,
                                C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "dk_level_fields": (C.c_int, [C.c_void_p, C.POINTER(dk_problem), C.c_int32, C.c_int32, C.c_uint64, C.c_uint64,
                                  C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dk_alg1_host": (C.c_int, [C.c_double, C.c_int32, C.POINTER(C.c_double), C.POINTER(dk_mlmc_opts), SAMPLER,
                               C.c_void_p, C.POINTER(dk_mlmc_result)]),
    "dk_cnn_init": (C.c_int, [C.c_uint64, C.POINTER(C.c_float)]),
    "dk_cnn_forward": (C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    "dk_cnn_loss_grad": (C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.POINTER(C.c_float), C.POINTER(C.c_double), C.c_void_p]),
    "dk_cv_train": (C.c_int, [C.c_void_p, C.POINTER(dk_problem), C.c_int32, C.c_uint64, C.c_int32, C.c_int32,
                              C.c_double, C.c_uint64, C.POINTER(C.c_float), C.POINTER(C.c_double),
                              C.POINTER(C.c_double), C.c_void_p]),
    "dk_context_stats": (C.c_int, [C.c_void_p, C.POINTER(dk_kernel_stats), C.c_int32]),
    "dk_context_reset": (C.c_int, [C.c_void_p, C.c_int32]),
    "dk_context_set_shape": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "dk_shape_rows": (C.c_int, [C.c_int32, C.c_int32]),
    "dk_shape_spw": (C.c_int, [C.c_int32, C.c_int32]),
    "dk_context_set_launch_cap": (C.c_int, [C.c_void_p, C.c_double]),
    "dk_context_tuning_json": (C.c_int, [C.c_void_p, C.c_char_p, C.c_uint64]),
    "dk_context_load_tuning_json": (C.c_int, [C.c_void_p, C.c_char_p]),
    "dk_context_set_streaming": (C.c_int, [C.c_void_p, C.c_int32]),
    "dk_context_set_stream_depth": (C.c_int, [C.c_void_p, C.c_int32]),
    "dk_heat_steps": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_void_p, C.c_void_p,
                                C.POINTER(C.c_double), C.c_void_p]),
    "dk_last_error": (C.c_char_p, []),
    "dk_version": (C.c_char_p, []),
    "dk_abi_sizes": (C.c_int, [C.POINTER(C.c_int32), C.c_int32]),
}

_lib = None


def load():
    """Load libdk_mlmc.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                           "or `python paper_2311_08872_amd/build.py`")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    sizes = (C.c_int32 * 16)()
    k = L.dk_abi_sizes(sizes, 16)
    mine = [C.sizeof(t) for t in (dk_mode, dk_field, dk_obs, dk_problem, dk_moments, dk_mlmc_opts, dk_mlmc_result,
                                  dk_kernel_stats)]
    if list(sizes[:k]) != mine:
        raise RuntimeError(f"ABI mismatch between include/dk_mlmc.h ({list(sizes[:k])}) and the binding ({mine})")
    _lib = L
    return L
