"""ctypes declarations of the C ABI in include/rsv_hmc.h.

Loads the in-tree HIP library ``librsvhmc.so``.  There is no fallback: if the
library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librsvhmc.so")

RSV_OK, RSV_EINVAL, RSV_EDEVICE, RSV_ENOMEM, RSV_ESTATE, RSV_ENONFINITE = 0, -1, -2, -3, -4, -5
RSV_F64, RSV_F32_MIXED = 0, 1
RSV_TERM_RETURN, RSV_TERM_RV, RSV_TERMS_RSV = 1, 2, 3
RSV_FLAG_RESIDENT = 1
RSV_FLAG_LEVEL_MOVE = 2
RSV_FLAG_OMELYAN = 4
RSV_FLAG_FOREST_RUTH = 8
RSV_STATIC_WORKSPACE_BYTES = 32 << 20

THETA_KEYS = ("phi", "mu", "xi", "sig2_eta", "sig2_u")
PRIOR_KEYS = ("mu_mean", "mu_var", "xi_mean", "xi_var",
              "eta_shape", "eta_scale", "u_shape", "u_scale")

# Every symbol include/rsv_hmc.h declares.
EXPORTS = ("rsv_hmc_workspace_bytes", "rsv_hmc_state_size", "rsv_hmc_init",
           "rsv_hmc_init_static", "rsv_hmc_momenta",
           "rsv_hmc_trajectory", "rsv_theta_update", "rsv_hmc_sweep", "rsv_hmc_check",
           "rsv_hmc_profile", "rsv_hmc_kernel_time", "rsv_hmc_destroy", "rsv_last_error",
           "rsv_mlp_features", "rsv_mlp_forward", "rsv_mlp_grad_workspace_bytes", "rsv_mlp_grad",
           "rsv_mlp_adam")
MLP_INPUTS, MLP_INPUTS_PAD, MLP_HIDDEN, MLP_PARAMS = 27, 32, 64, 6337


class rsv_theta(C.Structure):
    _fields_ = [(k, C.c_double) for k in THETA_KEYS]


class rsv_prior(C.Structure):
    _fields_ = [(k, C.c_double) for k in PRIOR_KEYS]


class rsv_leapfrog(C.Structure):
    _fields_ = [("n_steps", C.c_int32), ("reserved", C.c_int32), ("dtau", C.c_double)]


class rsv_problem(C.Structure):
    _fields_ = [
        ("n_series", C.c_int32),
        ("chains_per_series", C.c_int32),
        ("offsets", C.POINTER(C.c_int64)),
        ("y", C.c_void_p),
        ("log_rv", C.c_void_p),
        ("precision", C.c_int32),
        ("terms", C.c_int32),
        ("max_steps", C.c_int32),
        ("sites_per_lane", C.c_int32),
        ("waves_per_tile", C.c_int32),
        ("flags", C.c_int32),
        ("seed", C.c_uint64),
        ("dtau_jitter", C.c_double),
        ("prior", rsv_prior),
    ]


class rsv_trace(C.Structure):
    _fields_ = [("delta_h", C.c_void_p), ("accepted", C.c_void_p), ("theta", C.c_void_p),
                ("h", C.c_void_p), ("h_batch_sum", C.c_void_p), ("h_sq_sum", C.c_void_p),
                ("batch_len", C.c_int32), ("reserved", C.c_int32)]


def load(path: str | None = None) -> C.CDLL:
    """The HIP library at `path`, by default the module's LIB_PATH as it is
    at the call (a caller may point LIB_PATH at another build first)."""
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(
            f"HIP library {path} is not built; run `python -m paper_1603_08114_amd.build` "
            "(or __graft_entry__.build()) first")
    lib = C.CDLL(path)
    P, V = C.POINTER, C.c_void_p
    sig = {
        "rsv_hmc_workspace_bytes": (C.c_size_t, [P(rsv_problem)]),
        "rsv_hmc_state_size": (C.c_int64, [P(rsv_problem)]),
        "rsv_hmc_init": (C.c_int32, [P(V), P(rsv_problem), V, V, V, V, C.c_size_t, V]),
        "rsv_hmc_init_static": (C.c_int32, [P(V), P(rsv_problem), V, V, V, V]),
        "rsv_hmc_momenta": (C.c_int32, [V, C.c_uint64, V]),
        "rsv_hmc_trajectory": (C.c_int32, [V, C.c_uint64, P(rsv_leapfrog), V, V, V, V]),
        "rsv_theta_update": (C.c_int32, [V, C.c_uint64, V]),
        "rsv_hmc_sweep": (C.c_int32, [V, C.c_uint64, C.c_int32, P(rsv_leapfrog), C.c_int32,
                                      P(rsv_trace)]),
        "rsv_hmc_check": (C.c_int32, [V, P(C.c_int64)]),
        "rsv_hmc_profile": (C.c_int32, [V, C.c_int32]),
        "rsv_hmc_kernel_time": (C.c_int32, [V, P(C.c_double), P(C.c_int64)]),
        "rsv_hmc_destroy": (C.c_int32, [V]),
        "rsv_last_error": (C.c_char_p, []),
        "rsv_mlp_features": (C.c_int32, [C.c_int32, V, V, V, V, V, V, C.c_int64, V, V]),
        "rsv_mlp_forward": (C.c_int32, [C.c_int64, V, V, V, C.c_int32, V]),
        "rsv_mlp_grad_workspace_bytes": (C.c_size_t, [C.c_int64]),
        "rsv_mlp_grad": (C.c_int32, [C.c_int64, V, V, V, V, V, V, V, C.c_size_t, V]),
        "rsv_mlp_adam": (C.c_int32, [V, V, V, V, C.c_int32, C.c_float, C.c_float, C.c_float,
                                     C.c_float, V]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib
