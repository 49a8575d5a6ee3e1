"""ctypes declarations of the libgld C ABI (include/gld.h), same names.

Argument marshalling only: every step of the integrator runs in the HIP
kernels of libgld.so.  Importing this module fails loudly when the library
has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgld.so")

GLD_OK = 0
GLD_ERR_INVALID_ARG = -1
GLD_ERR_NOT_PD = -2
GLD_ERR_NO_CONV = -3
GLD_ERR_NONFINITE = -4
GLD_ERR_OOM = -5
GLD_ERR_DEVICE = -6
GLD_ERR_BOX = -7
GLD_ERR_CAPACITY = -8
GLD_ERR_INTERVAL = -9

GLD_FP64 = 0
GLD_FP32_MIXED = 1
GLD_PAIR_ISOTROPIC = 0
GLD_PAIR_PARALLEL = 1

(GLD_K_HISTORY, GLD_K_DISSIPATIVE, GLD_K_NOISE_FIR, GLD_K_NOISE_SPMV, GLD_K_UPDATE, GLD_K_NEIGHBOR,
 GLD_K_CHECK, GLD_K_NOISE_SETUP, GLD_K_COUNT) = range(9)
KERNEL_NAMES = ["history", "dissipative", "noise_fir", "noise_spmv", "update", "neighbor", "check", "noise_setup"]

_dp = C.POINTER(C.c_double)


class gld_params(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("box", C.c_double * 3),
        ("dt", C.c_double),
        ("mass", C.c_double),
        ("kT", C.c_double),
        ("m_max", C.c_int32),
        ("n_r", C.c_int32),
        ("k_self", _dp),
        ("k_pair_g", _dp),
        ("k_pair_w", _dp),
        ("r0", C.c_double),
        ("dr", C.c_double),
        ("r_cut", C.c_double),
        ("r_cut_min", C.c_double),
        ("pair_tensor", C.c_int32),
        ("precision", C.c_int32),
        ("wca_sigma", C.c_double),
        ("wca_eps", C.c_double),
        ("seed", C.c_uint64),
        ("noise_tol", C.c_double),
        ("lam_lo", C.c_double),
        ("lam_hi", C.c_double),
        ("max_neighbors", C.c_int32),
        ("check_interval", C.c_int32),
        ("verlet_skin", C.c_double),
        ("noise_window", C.c_int32),
        ("k_pair", _dp),
        ("dk_self", _dp),
        ("noise_a", _dp),
        ("noise_b", _dp),
        ("noise_rank", C.c_int32),
        ("noise_terms", C.c_int32),
        ("check_iters", C.c_int32),
        ("rebuild_period", C.c_int32),
    ]


class gld_state(C.Structure):
    _fields_ = [
        ("r", _dp),
        ("v", _dp),
        ("f_c", _dp),
        ("f_d", _dp),
        ("f_r", _dp),
        ("history", _dp),
        ("step", C.c_int64),
        ("flags", C.c_int32),
        ("flag_step", C.c_int64),
    ]


class gld_noise_info(C.Structure):
    _fields_ = [
        ("cheb_terms", C.c_int32),
        ("rank", C.c_int32),
        ("block", C.c_int32),
        ("lam_lo", C.c_double),
        ("lam_hi", C.c_double),
        ("lam_singular", C.c_double),
        ("err_estimate", C.c_double),
        ("window_half", C.c_int32),
        ("noise_window", C.c_int32),
        ("cheb_terms_tight", C.c_int32),
        ("lam_hi_tight", C.c_double),
        ("lam_lo_tight", C.c_double),
        ("tight_steps", C.c_int64),
        ("list_index_bits", C.c_int32),
        ("theta_min", C.c_double),
        ("theta_max", C.c_double),
        ("tight_retired", C.c_int32),
        ("filters_given", C.c_int32),
        ("list_weight_bits", C.c_int32),
    ]


EXPORTED = [
    "gld_workspace_size", "gld_create", "gld_step", "gld_sync", "gld_read_state", "gld_write_state",
    "gld_noise_parameters", "gld_set_graph", "gld_set_timing", "gld_kernel_times", "gld_destroy",
    "gld_white_noise", "gld_build_noise_filters", "gld_status_string", "gld_last_error", "gld_create_static",
    "gld_list_stats",
]

GLD_STATIC_WORKSPACE_BYTES = 64 << 20

# include/gld_batch.h
EXPORTED_BATCH = [
    "gld_batch_base_size", "gld_batch_create", "gld_batch_footprint", "gld_batch_add", "gld_batch_remove",
    "gld_batch_step", "gld_batch_sync", "gld_batch_read_state", "gld_batch_write_state",
    "gld_batch_noise_parameters", "gld_batch_autotune", "gld_batch_set_schedule", "gld_batch_stats",
    "gld_batch_destroy", "gld_batch_set_timing", "gld_batch_kernel_times", "gld_batch_system_stats",
]
GLD_BATCH_CANDIDATES = 8

# include/gld_serve.h
EXPORTED_SERVE = [
    "gld_server_create", "gld_server_submit", "gld_server_run", "gld_server_request", "gld_server_stats",
    "gld_server_destroy",
]


# include/gld_general.h
EXPORTED_GENERAL = [
    "gld_general_workspace_size", "gld_general_create", "gld_general_step", "gld_general_sync",
    "gld_general_read_state", "gld_general_write_state", "gld_general_frequency_vectors", "gld_general_get_info",
    "gld_general_set_timing", "gld_general_kernel_times", "gld_general_destroy",
]
GLD_GENERAL_MAX_N = 32768
GLD_GENERAL_MAX_ITERS = 128
GENERAL_KERNEL_NAMES = ["dissipative", "dft", "lanczos", "combine", "pairs", "update"]
GLD_G_COUNT = len(GENERAL_KERNEL_NAMES)


class gld_general_info(C.Structure):
    _fields_ = [
        ("max_iters", C.c_int32),
        ("last_iters", C.c_int32),
        ("pairs", C.c_int64),
        ("max_per_particle", C.c_int32),
        ("capacity", C.c_int32),
        ("tol", C.c_double),
    ]


class gld_request_info(C.Structure):
    _fields_ = [
        ("id", C.c_int64),
        ("n", C.c_int64),
        ("m_max", C.c_int32),
        ("status", C.c_int32),
        ("steps", C.c_int64),
        ("footprint", C.c_size_t),
        ("arrival_s", C.c_double),
        ("admitted_s", C.c_double),
        ("done_s", C.c_double),
    ]


class gld_batch_schedule(C.Structure):
    _fields_ = [("lanes_threshold", C.c_int32 * 3)]


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libgld.so not built at {path}; run __graft_entry__.build() "
                          "(there is no fallback implementation)")
    lib = C.CDLL(path)
    vp = C.c_void_p
    P = C.POINTER(gld_params)
    S = C.POINTER(gld_state)
    lib.gld_workspace_size.argtypes = [P, C.POINTER(C.c_size_t)]
    lib.gld_create.argtypes = [P, _dp, _dp, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.gld_create_static.argtypes = [P, _dp, _dp, vp, C.POINTER(vp)]
    lib.gld_step.argtypes = [vp, C.c_int64]
    lib.gld_sync.argtypes = [vp]
    lib.gld_read_state.argtypes = [vp, S]
    lib.gld_write_state.argtypes = [vp, S]
    lib.gld_noise_parameters.argtypes = [vp, C.POINTER(gld_noise_info)]
    lib.gld_set_graph.argtypes = [vp, C.c_int]
    lib.gld_list_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    lib.gld_set_timing.argtypes = [vp, C.c_int]
    lib.gld_kernel_times.argtypes = [vp, _dp, C.POINTER(C.c_int64)]
    lib.gld_destroy.argtypes = [vp]
    lib.gld_white_noise.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int64, vp, vp, vp]
    lib.gld_build_noise_filters.argtypes = [P, C.c_double, C.c_double, C.c_double, _dp, C.c_size_t, _dp,
                                            C.c_size_t, C.POINTER(gld_noise_info)]
    PP = C.POINTER(P)
    dpp = C.POINTER(_dp)
    lib.gld_batch_base_size.argtypes = [C.c_int32, C.POINTER(C.c_size_t)]
    lib.gld_batch_create.argtypes = [C.c_int32, C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.gld_batch_footprint.argtypes = [vp, P, _dp, C.POINTER(C.c_size_t)]
    lib.gld_batch_add.argtypes = [vp, C.c_int32, PP, dpp, dpp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.gld_batch_remove.argtypes = [vp, C.c_int32]
    lib.gld_batch_step.argtypes = [vp, C.c_int64]
    lib.gld_batch_sync.argtypes = [vp]
    lib.gld_batch_read_state.argtypes = [vp, C.c_int32, S]
    lib.gld_batch_write_state.argtypes = [vp, C.c_int32, S]
    lib.gld_batch_noise_parameters.argtypes = [vp, C.c_int32, C.POINTER(gld_noise_info)]
    lib.gld_batch_autotune.argtypes = [vp, C.c_int32, C.POINTER(gld_batch_schedule), _dp]
    lib.gld_batch_set_schedule.argtypes = [vp, C.POINTER(gld_batch_schedule)]
    lib.gld_batch_stats.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.gld_batch_destroy.argtypes = [vp]
    lib.gld_batch_system_stats.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    lib.gld_batch_set_timing.argtypes = [vp, C.c_int]
    lib.gld_batch_kernel_times.argtypes = [vp, _dp, C.POINTER(C.c_int64)]
    for name in EXPORTED_BATCH:
        getattr(lib, name).restype = C.c_int
    lib.gld_server_create.argtypes = [C.c_int32, C.c_int32, vp, C.c_size_t, vp, C.c_int32,
                                      C.POINTER(gld_batch_schedule), C.POINTER(vp)]
    lib.gld_server_submit.argtypes = [vp, P, _dp, _dp, C.c_int64, C.c_double, C.POINTER(C.c_int64),
                                      C.POINTER(C.c_size_t)]
    lib.gld_server_run.argtypes = [vp]
    lib.gld_server_request.argtypes = [vp, C.c_int64, C.POINTER(gld_request_info), S]
    lib.gld_server_stats.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.gld_server_destroy.argtypes = [vp]
    for name in EXPORTED_SERVE:
        getattr(lib, name).restype = C.c_int
    lib.gld_general_workspace_size.argtypes = [P, C.c_int32, C.POINTER(C.c_size_t)]
    lib.gld_general_create.argtypes = [P, C.c_int32, _dp, _dp, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.gld_general_step.argtypes = [vp, C.c_int64]
    lib.gld_general_sync.argtypes = [vp]
    lib.gld_general_read_state.argtypes = [vp, S]
    lib.gld_general_write_state.argtypes = [vp, S]
    lib.gld_general_frequency_vectors.argtypes = [vp, C.c_int32, C.c_int32, _dp]
    lib.gld_general_get_info.argtypes = [vp, C.POINTER(gld_general_info)]
    lib.gld_general_set_timing.argtypes = [vp, C.c_int]
    lib.gld_general_kernel_times.argtypes = [vp, _dp, C.POINTER(C.c_int64)]
    lib.gld_general_destroy.argtypes = [vp]
    for name in EXPORTED_GENERAL:
        getattr(lib, name).restype = C.c_int
    lib.gld_status_string.restype = C.c_char_p
    lib.gld_status_string.argtypes = [C.c_int]
    lib.gld_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("gld_status_string", "gld_last_error"):
            getattr(lib, name).restype = C.c_int
    return lib
