"""ctypes declarations of the C ABI in include/lindblad.h, lindblad_serve.h and
lindblad_kernels.h.

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation of any part of the step.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblindblad.so")

LB_MAX_MODES = 8
LB_MAX_SITES = 64

LB_OK, LB_ERR_ARG, LB_ERR_OOM, LB_ERR_HIP, LB_ERR_NUMERIC, LB_ERR_UNSTABLE, LB_ERR_STATE = \
    0, -1, -2, -3, -4, -5, -6
LB_WARN_UNSTABLE = 1
LB_FP64, LB_FP32_CONTRACT = 0, 1

FACTOR_KINDS = {"ID": 0, "A_POW": 1, "ADAG_POW": 2, "ADAG_A": 3, "NUM_POW": 4,
                "CHARGE_POW": 5, "SHIFT": 6, "DENSE": 7}

EXPORTED = ["lindblad_default_config", "lindblad_create", "lindblad_destroy",
            "lindblad_mpo_build", "lindblad_op_info", "lindblad_op_site", "lindblad_set_generator",
            "lindblad_kraus_info", "lindblad_kraus_site", "lindblad_set_state_product", "lindblad_set_state_mps",
            "lindblad_get_state_mps", "lindblad_restore_state", "lindblad_step", "lindblad_sync", "lindblad_step_batch",
            "lindblad_observe", "lindblad_trace_purity", "lindblad_diagnostics",
            "lindblad_last_error", "lindblad_profile", "lindblad_profile_mask", "lindblad_profile_read", "lindblad_kernel_zgemm", "lindblad_kernel_heev",
            "lindblad_kernel_truncate", "lindblad_kernel_set_wait_limit", "lindblad_kernel_heev_noalloc", "lindblad_get_config", "lindblad_footprint", "lindblad_release",
            "lindblad_server_create", "lindblad_server_submit", "lindblad_server_run",
            "lindblad_server_result", "lindblad_server_stats", "lindblad_server_destroy",
            "lindblad_gemm_tune_save", "lindblad_gemm_tune_load", "lindblad_gemm_tune_entries"]


class LbConfig(C.Structure):
    _fields_ = [("n_modes", C.c_int32), ("bits", C.c_int32 * LB_MAX_MODES),
                ("n_sites", C.c_int32), ("site_order", (C.c_int32 * 2) * LB_MAX_SITES),
                ("chi_cap", C.c_int32), ("chi_mu_cap", C.c_int32), ("chi_zip_cap", C.c_int32),
                ("tol", C.c_double), ("tol_zip", C.c_double), ("order", C.c_int32),
                ("precision", C.c_int32), ("allow_unstable", C.c_int32),
                ("stream", C.c_void_p), ("device", C.c_int32),
                ("fp32_tol_floor", C.c_double), ("tau_warn", C.c_double),
                ("arena", C.c_void_p), ("arena_bytes", C.c_int64),
                ("fixed_bounds", C.c_int32), ("fp64_jacobi_pass", C.c_int32),
                ("autotune", C.c_int32)]


class LbFactor(C.Structure):
    _fields_ = [("mode", C.c_int32), ("kind", C.c_int32), ("p", C.c_int32), ("q", C.c_int32),
                ("offset", C.c_int64), ("dense", C.POINTER(C.c_double))]


class LbTerm(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double), ("n_factors", C.c_int32),
                ("factors", C.POINTER(LbFactor))]


class LbDrive(C.Structure):
    _fields_ = [("n", C.c_int32), ("coef", C.POINTER(C.c_double)),
                ("omega", C.POINTER(C.c_double)), ("phase", C.POINTER(C.c_double))]


class LbDiag(C.Structure):
    _fields_ = [("steps", C.c_int64), ("t", C.c_double), ("tau", C.c_double),
                ("max_tau_defect", C.c_double), ("n_sites", C.c_int32),
                ("bonds", C.c_int32 * LB_MAX_SITES), ("chi_mu", C.c_int32),
                ("zip_bonds", C.c_int32 * LB_MAX_SITES),
                ("discarded", C.c_double * LB_MAX_SITES), ("tier", C.c_int32),
                ("bound_redos", C.c_int64)]


class LbProfile(C.Structure):
    _fields_ = [("n", C.c_int32), ("name", (C.c_char * 24) * 16), ("launches", C.c_int64 * 16),
                ("ms", C.c_double * 16), ("flop", C.c_double * 16), ("bytes", C.c_double * 16)]


class LbServerConfig(C.Structure):
    _fields_ = [("n_slots", C.c_int32), ("hbm_budget", C.c_int64)]


class LbRequest(C.Structure):
    _fields_ = [("solver", C.c_void_p), ("init", C.POINTER(C.POINTER(C.c_double))),
                ("n_steps", C.c_int32), ("obs", C.POINTER(C.c_void_p)), ("n_obs", C.c_int32),
                ("arrival", C.c_double)]


class LbResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("arrival", C.c_double), ("admitted", C.c_double),
                ("done", C.c_double), ("bytes", C.c_int64), ("max_tau_defect", C.c_double),
                ("chi_mu", C.c_int32), ("max_bond", C.c_int32)]


class LbServerStats(C.Structure):
    _fields_ = [("makespan", C.c_double), ("peak_bytes", C.c_int64), ("peak_running", C.c_int32),
                ("completed", C.c_int32)]


_lib = None


def lib_path() -> str:
    return LIB_PATH


def load() -> C.CDLL:
    """Load liblindblad.so (built by paper_2605_27515_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with `python -m paper_2605_27515_amd.build`"
                           " (the GPU path has no fallback)")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.lindblad_default_config.argtypes = [C.POINTER(LbConfig)]
    lib.lindblad_default_config.restype = None
    lib.lindblad_create.argtypes = [C.POINTER(LbConfig), C.POINTER(vp)]
    lib.lindblad_destroy.argtypes = [vp]
    lib.lindblad_destroy.restype = None
    lib.lindblad_mpo_build.argtypes = [vp, C.POINTER(LbTerm), C.c_int32, C.c_double, C.POINTER(vp)]
    lib.lindblad_op_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.lindblad_op_site.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double)]
    lib.lindblad_kraus_site.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_double)]
    lib.lindblad_set_generator.argtypes = [vp, vp, vp, C.POINTER(LbDrive), C.POINTER(vp), C.c_int32,
                                           C.c_double]
    lib.lindblad_kraus_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.lindblad_set_state_product.argtypes = [vp, C.POINTER(C.POINTER(C.c_double))]
    lib.lindblad_set_state_mps.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.POINTER(C.c_double))]
    lib.lindblad_get_state_mps.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.POINTER(C.c_double))]
    lib.lindblad_restore_state.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.POINTER(C.c_double)), C.c_int64]
    lib.lindblad_step.argtypes = [vp, C.c_int32]
    lib.lindblad_sync.argtypes = [vp]
    lib.lindblad_step_batch.argtypes = [C.POINTER(vp), C.c_int32, C.c_int32]
    lib.lindblad_observe.argtypes = [vp, vp, C.POINTER(C.c_double)]
    lib.lindblad_trace_purity.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.lindblad_diagnostics.argtypes = [vp, C.POINTER(LbDiag)]
    lib.lindblad_gemm_tune_save.argtypes = [C.c_char_p]
    lib.lindblad_gemm_tune_load.argtypes = [C.c_char_p]
    lib.lindblad_gemm_tune_entries.argtypes = []
    lib.lindblad_gemm_tune_entries.restype = C.c_int64
    dp = C.POINTER(C.c_double)
    lib.lindblad_kernel_zgemm.argtypes = [C.c_int32, C.c_int32, C.c_int32, dp, C.c_int32, dp, C.c_int32,
                                          dp, C.c_int32, C.c_int32]
    lib.lindblad_kernel_heev.argtypes = [C.c_int32, dp, dp, dp, C.POINTER(C.c_int32), C.c_int32]
    lib.lindblad_kernel_heev_noalloc.argtypes = [C.c_int32, vp, vp, vp, C.POINTER(C.c_int32), C.c_int32, vp]
    lib.lindblad_kernel_truncate.argtypes = [C.c_int32, dp, C.c_double, C.c_int32, C.POINTER(C.c_int32), dp]
    lib.lindblad_kernel_set_wait_limit.argtypes = [C.c_int64]
    lib.lindblad_profile.argtypes = [vp, C.c_int32]
    lib.lindblad_profile_mask.argtypes = [vp, C.c_uint32]
    lib.lindblad_profile_read.argtypes = [vp, C.POINTER(LbProfile)]
    lib.lindblad_get_config.argtypes = [vp, C.POINTER(LbConfig)]
    lib.lindblad_footprint.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.lindblad_release.argtypes = [vp]
    lib.lindblad_server_create.argtypes = [C.POINTER(LbServerConfig), C.POINTER(vp)]
    lib.lindblad_server_submit.argtypes = [vp, C.POINTER(LbRequest), C.POINTER(C.c_int32)]
    lib.lindblad_server_run.argtypes = [vp]
    lib.lindblad_server_result.argtypes = [vp, C.c_int32, C.POINTER(LbResult), C.POINTER(C.c_double)]
    lib.lindblad_server_stats.argtypes = [vp, C.POINTER(LbServerStats)]
    lib.lindblad_server_destroy.argtypes = [vp]
    lib.lindblad_server_destroy.restype = None
    lib.lindblad_last_error.argtypes = []
    lib.lindblad_last_error.restype = C.c_char_p
    for name in EXPORTED:
        fn = getattr(lib, name)
        if name not in ("lindblad_default_config", "lindblad_destroy", "lindblad_last_error",
                        "lindblad_server_destroy", "lindblad_gemm_tune_entries"):
            fn.restype = C.c_int
    _lib = lib
    return lib
