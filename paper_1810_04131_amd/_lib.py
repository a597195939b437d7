"""ctypes declarations of the C ABI in include/yqbx.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libyqbx.so")

YQ_OK = 0
YQ_EINVAL = -1
YQ_EGEOM = -2
YQ_ENOCONV = -3
YQ_ENOMEM = -4
YQ_EDEVICE = -5
YQ_ESTATE = -6
YQ_EADMIT = -7
YQ_FP64 = 0
YQ_MIXED = 1
YQ_FMM64 = 2
YQ_FAR_DIRECT = 0
YQ_FAR_FMM = 1
YQ_FAR_AUTO = 2
YQ_FAR_CUTOFF = 3
YQ_LABEL_ARC = 0
YQ_LABEL_JANUS = 1
YQ_M2L_MFMA = 0
YQ_M2L_VALU = 1
YQ_M2L_MFMA64 = 2

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
c_char_p = ctypes.c_char_p


class yq_params(ctypes.Structure):
    _fields_ = [
        ("panels_per_particle", c_int32),
        ("qbx_order", c_int32),
        ("qbx_window", c_int32),
        ("qbx_oversample", c_int32),
        ("qbx_radius", c_double),
        ("near_beta", c_double),
        ("near_oversample", c_int32),
        ("pot_oversample", c_int32),
        ("pot_beta", c_double),
        ("precision", c_int32),
        ("far_mode", c_int32),
        ("fmm_order", c_int32),
        ("fmm_leaf_max", c_int32),
        ("tol", c_double),
        ("maxiter", c_int32),
        ("restart", c_int32),
        ("inner_tol", c_double),
        ("max_refine", c_int32),
        ("fmm_resid_order", c_int32),
        ("fmm_m2l", c_int32),
        ("cutoff_tol", c_double),
        ("sl_coupling", c_double),
        ("refine_levels", c_int32),
        ("refine_ratio", c_double),
    ]


class yq_solve_info(ctypes.Structure):
    _fields_ = [
        ("iterations", c_int32),
        ("outer_steps", c_int32),
        ("matvecs_fp64", c_int32),
        ("matvecs_fp32", c_int32),
        ("residual", c_double),
        ("seconds", c_double),
    ]


class yq_dynamics(ctypes.Structure):
    _fields_ = [
        ("dt", c_double),
        ("xi_x", c_double),
        ("xi_theta", c_double),
        ("gamma", c_double),
        ("c0", c_double),
        ("q", c_int32),
    ]


P = c_void_p  # opaque pointers (problem handles, device pointers)

SIGNATURES = {
    "yq_default_params": (None, [ctypes.POINTER(yq_params)]),
    "yq_create": (c_int32, [ctypes.POINTER(yq_params), ctypes.POINTER(c_void_p)]),
    "yq_destroy": (None, [P]),
    "yq_error_string": (c_char_p, [c_int32]),
    "yq_last_error": (c_char_p, [P]),
    "yq_set_stream": (c_int32, [P, P]),
    "yq_set_particles": (c_int32, [P, c_int32, P, P, P, c_double]),
    "yq_num_nodes": (c_int32, [P, ctypes.POINTER(c_int64)]),
    "yq_num_particles": (c_int32, [P, ctypes.POINTER(c_int32)]),
    "yq_get_nodes": (c_int32, [P, P, P, P, P, P]),
    "yq_near_count": (c_int32, [P, ctypes.POINTER(c_int64)]),
    "yq_get_near": (c_int32, [P, P, P]),
    "yq_boundary_label": (c_int32, [P, c_int32, c_double, c_double, P]),
    "yq_set_boundary_data": (c_int32, [P, P]),
    "yq_apply_far": (c_int32, [P, P, P, c_int32]),
    "yq_apply_operator": (c_int32, [P, P, P, c_int32]),
    "yq_solve": (c_int32, [P, P, P, ctypes.POINTER(yq_solve_info)]),
    "yq_surface_gradient": (c_int32, [P, P, P, P]),
    "yq_forces": (c_int32, [P, P, c_double, P, P, ctypes.POINTER(c_double)]),
    "yq_solve_forces": (c_int32, [P, P, P, ctypes.POINTER(yq_solve_info), c_double, P, P,
                                  ctypes.POINTER(c_double)]),
    "yq_eval_potential": (c_int32, [P, P, c_int64, P, P, P]),
    "yq_eval_potential_noalloc": (c_int32, [P, P, c_int64, P, P, P]),
    "yq_repulsion": (c_int32, [P, c_double, c_int32, P, P, ctypes.POINTER(c_double)]),
    "yq_step": (c_int32, [P, ctypes.POINTER(yq_dynamics), P, P, ctypes.POINTER(yq_solve_info), P,
                          P, P]),
    "yq_get_particles": (c_int32, [P, P, P]),
    "yq_bessel": (c_int32, [c_int32, c_int32, c_int32, c_int64, P, P]),
    "yq_fmm_stats": (c_int32, [P, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                               ctypes.POINTER(c_int32), ctypes.POINTER(c_double),
                               ctypes.POINTER(c_double)]),
    "yq_batch_create": (c_int32, [ctypes.POINTER(yq_params), ctypes.POINTER(c_void_p)]),
    "yq_batch_destroy": (None, [P]),
    "yq_batch_last_error": (c_char_p, [P]),
    "yq_batch_set_fmm": (c_int32, [P, c_int64, c_int32]),
    "yq_batch_set_fmm_engine": (c_int32, [P, c_int32]),
    "yq_batch_set_symmetric_far": (c_int32, [P, c_int32]),
    "yq_batch_set_near_cache": (c_int32, [P, c_int64]),
    "yq_batch_near_cache_info": (c_int32, [P, ctypes.POINTER(c_int64), ctypes.POINTER(c_int32),
                                           ctypes.POINTER(c_int32)]),
    "yq_batch_set_configs": (c_int32, [P, c_int32, P, P, P, P, P]),
    "yq_batch_num_nodes": (c_int32, [P, ctypes.POINTER(c_int64), P]),
    "yq_batch_boundary_label": (c_int32, [P, c_int32, c_double, c_double, P]),
    "yq_batch_set_boundary_data": (c_int32, [P, P]),
    "yq_batch_apply_operator": (c_int32, [P, P, P, c_int32]),
    "yq_batch_solve": (c_int32, [P, P, P]),
    "yq_batch_solve_forces": (c_int32, [P, P, P, c_double, P, P, P]),
    "yq_batch_forces": (c_int32, [P, P, c_double, P, P, P]),
    "yq_batch_autotune": (c_int32, [P, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32)]),
    "yq_batch_use_graphs": (c_int32, [P, c_int32]),
    "yq_batch_profile_enable": (c_int32, [P, c_int32]),
    "yq_batch_profile_read": (c_int32, [P, c_int32, ctypes.POINTER(c_int64), ctypes.POINTER(c_double),
                                        ctypes.POINTER(c_double), c_int32]),
    "yq_batch_profile_read_leaf": (c_int32, [P, c_int32, ctypes.POINTER(c_int64),
                                             ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                             ctypes.POINTER(c_double), c_int32]),
    "yq_server_create": (c_int32, [ctypes.POINTER(yq_params), c_int64, c_int32, c_double,
                                   ctypes.POINTER(c_void_p)]),
    "yq_server_destroy": (None, [P]),
    "yq_server_last_error": (c_char_p, [P]),
    "yq_server_set_fmm": (c_int32, [P, c_int64, c_int32]),
    "yq_server_submit": (c_int32, [P, c_int32, P, P, P, c_double, c_int32, c_double, c_double,
                                   ctypes.POINTER(c_int64)]),
    "yq_server_step": (c_int32, [P, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                                 ctypes.POINTER(c_int32)]),
    "yq_server_result": (c_int32, [P, c_int64, ctypes.POINTER(c_int32), ctypes.POINTER(c_int64),
                                   ctypes.POINTER(c_int32), P, P, P, ctypes.POINTER(c_double),
                                   ctypes.POINTER(yq_solve_info), ctypes.POINTER(c_double)]),
    "yq_server_release": (c_int32, [P, c_int64]),
    "yq_server_cancel": (c_int32, [P, c_int64]),
    "yq_profile_enable": (c_int32, [P, c_int32]),
    "yq_profile_read": (c_int32, [P, c_int32, ctypes.POINTER(c_int64), ctypes.POINTER(c_double),
                                  c_int32]),
}

_lib = None


class YQError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def load():
    """Loads libyqbx.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1810_04131_amd/build.py")
    # The library must run on PyTorch's HIP runtime, whose tensors and streams it
    # is handed: with torch's runtime mapped first, the library's dependency on
    # libamdhip64 resolves to it.  Opened first, it would pull in a second HIP
    # and HSA runtime next to torch's, and device allocations fail.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, handle=None, batch=False, server=False):
    if status == YQ_OK:
        return status
    lib = load()
    if server:
        detail = lib.yq_server_last_error(handle)
    elif batch:
        detail = lib.yq_batch_last_error(handle)
    else:
        detail = lib.yq_last_error(handle)
    detail = detail.decode() if detail else ""
    base = lib.yq_error_string(status).decode()
    raise YQError(status, f"{base}: {detail}")
