"""ctypes loader for libmrx.so (the HIP library built by ``build.py``).

There is no fallback: if the library is missing or fails to load, importing
the operators raises, so nothing can silently run on the CPU.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrx.so")

_lib = None

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_size_t = ctypes.c_size_t
c_uint32 = ctypes.c_uint32
c_float = ctypes.c_float
c_char_p = ctypes.c_char_p
c_void_p = ctypes.c_void_p
P = c_void_p  # device pointers, plan handles and streams

# name -> (restype, argtypes); every function declared in include/mrx.h.
SIGNATURES = {
    "mrx_version": (c_char_p, []),
    "mrx_last_error": (c_char_p, []),
    "mrx_plan_create": (c_int32, [ctypes.POINTER(c_void_p), c_int32, ctypes.POINTER(c_int32),
                                  ctypes.POINTER(c_int32), ctypes.POINTER(c_int32), c_uint32]),
    "mrx_plan_destroy": (None, [P]),
    "mrx_plan_sizes": (c_int32, [P, ctypes.POINTER(c_int64), ctypes.POINTER(c_int64), ctypes.POINTER(c_int64)]),
    "mrx_plan_workspace_bytes": (c_size_t, [P]),
    "mrx_plan_set_workspace": (c_int32, [P, P, c_size_t]),
    "mrx_supported_length": (c_int32, [c_int32]),
    "mrx_sense_fwd": (c_int32, [P, P, P, P, P, P, P]),
    "mrx_sense_adj": (c_int32, [P, P, P, P, P, P]),
    "mrx_sense_normal": (c_int32, [P, P, P, P, P, P, P]),
    "mrx_cg_dc": (c_int32, [P, P, P, P, P, P, c_int32, P, P, P]),
    "mrx_cg_dc_backward": (c_int32, [P, P, P, P, P, P, P, c_int32, P, P, P, c_int32, P]),
    "mrx_cg_dc_noalloc": (c_int32, [P, P, P, P, P, P, c_int32, P, P, P, P]),
    "mrx_soft_sense_fwd": (c_int32, [P, P, P, P, P, P, P]),
    "mrx_soft_sense_adj": (c_int32, [P, P, P, P, P, P]),
    "mrx_soft_sense_normal": (c_int32, [P, P, P, P, P, P, P]),
    "mrx_soft_cg_dc": (c_int32, [P, P, P, P, P, P, c_int32, P, P, P]),
    "mrx_soft_modl_forward": (c_int32, [P, P, P, P, P, c_int32, c_int32, P, P, P]),
    "mrx_soft_modl_backward": (c_int32, [P, P, P, P, P, P, P, c_int32, c_int32, P, P, P, c_int32, P]),
    "mrx_soft_coil_mse_grad": (c_int32, [P, P, P, P, P, P, P]),
    "mrx_ipalm_extrapolate": (c_int32, [P, P, P, c_int64, c_float, P]),
    "mrx_ipalm_update": (c_int32, [P, P, P, P, c_int64, c_float, P]),
    "mrx_vn_project": (c_int32, [P, c_int32, c_int32, P, c_int32, P]),
    "mrx_normalize_max": (c_int32, [P, P, P, P, P, P]),
    "mrx_sum_f32": (c_int32, [P, c_int32, P, c_int32, P]),
    "mrx_status_word": (c_int32, [P, P, c_int32, P]),
    "mrx_plan_autotune": (c_int32, [P, P, P, P, P, P]),
    "mrx_cnn_set_weights": (c_int32, [P, P, P]),
    "mrx_cnn_forward": (c_int32, [P, P, P, P]),
    "mrx_cnn_layer_forward": (c_int32, [P, c_int32, P, P, P]),
    "mrx_cnn_backward": (c_int32, [P, P, P, P, P, c_int32, P]),
    "mrx_modl_forward": (c_int32, [P, P, P, P, P, c_int32, c_int32, P, P, P]),
    "mrx_modl_forward_from": (c_int32, [P, P, P, P, P, P, c_int32, c_int32, P, P, P]),
    "mrx_cnn_set_bn": (c_int32, [P, P, P, P, P]),
    "mrx_nufft_fwd": (c_int32, [P, P, c_int32, P, P, P, P, P]),
    "mrx_nufft_adj": (c_int32, [P, P, c_int32, P, P, P, P]),
    "mrx_toeplitz_psf": (c_int32, [P, P, c_int32, P, P]),
    "mrx_toeplitz_supported": (c_int32, [c_int32]),
    "mrx_modl_backward": (c_int32, [P, P, P, P, P, P, P, c_int32, c_int32, P, P, P, c_int32, P]),
    "mrx_mse_grad": (c_int32, [P, P, P, P, P, P]),
    "mrx_adam_step": (c_int32, [P, P, P, P, c_int64, c_float, c_float, c_float, c_float, c_int32, P]),
    "mrx_plan_schedule": (c_char_p, [P, c_int32]),
    "mrx_plan_kernel_timing": (c_int32, [P, c_int32]),
    "mrx_plan_kernel_time": (c_int32, [P, c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(c_int32)]),
    "mrx_schedule_name": (c_char_p, [c_int32, c_int32]),
    "mrx_vn_stage": (c_int32, [P, P, P, P, P, P, P, P]),
    "mrx_vn_stage_backward": (c_int32, [P, P, P, P, P, P, P, P, P, P, P, c_int32, P]),
    "mrx_plan_set_schedule": (c_int32, [P, c_int32, c_char_p]),
    "mrx_dc_judge": (c_int32, [P, P, P, P, P, P, c_float, P, P, P]),
    "mrx_tune_cache_save": (c_int32, [c_char_p]),
    "mrx_tune_cache_load": (c_int32, [c_char_p, ctypes.POINTER(c_int32)]),
}

STATUS = {0: "MRX_OK", -1: "MRX_EINVAL", -2: "MRX_EUNSUPPORTED", -3: "MRX_ENOMEM",
          -4: "MRX_EHIP", -5: "MRX_ENOWORKSPACE"}


class CnnParams(ctypes.Structure):
    _fields_ = [("w", c_void_p * 5), ("b", c_void_p * 5)]


class VnParams(ctypes.Structure):
    _fields_ = [("k", c_void_p), ("w", c_void_p), ("lam", c_void_p)]


class CnnGrads(ctypes.Structure):
    _fields_ = [("w", c_void_p * 5), ("b", c_void_p * 5)]


class MrxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def lib():
    """Load libmrx.so once; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2202_14005_amd.build` "
            "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(code, what=""):
    if code != 0:
        msg = lib().mrx_last_error().decode(errors="replace")
        raise MrxError(code, f"{what}: {msg}" if what else msg)
