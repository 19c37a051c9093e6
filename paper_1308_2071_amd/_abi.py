"""ctypes binding of liblbmpm.so (include/lbm.h).  Argument marshalling only: every step of the
method runs in the library's HIP kernels.  Device buffers are torch tensors on a ROCm device;
the library works on torch's current HIP stream.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbmpm.so")

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_HIP = 0, -1, -2, -3
LBM_E_DIVERGED, LBM_E_STATE, LBM_E_UNSUPPORTED = -4, -5, -6
LBM_FP32, LBM_FP64, LBM_FP32_F64 = 0, 1, 2
LBM_LAYOUT_PULL, LBM_LAYOUT_AA = 0, 1
LBM_WALL_ISOTHERMAL, LBM_WALL_ADIABATIC, LBM_PERIODIC = 0, 1, 2
LBM_DIV_NONFINITE, LBM_DIV_SPEED, LBM_DIV_TEMPERATURE = 1, 2, 4


class LbmParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("bc", C.c_int32 * 4),
        ("T_wall", C.c_double * 4),
        ("Ra", C.c_double), ("Pr", C.c_double), ("Da", C.c_double), ("J", C.c_double),
        ("Ma", C.c_double), ("sigma", C.c_double), ("varpi", C.c_double), ("rho0", C.c_double),
        ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double),
        ("zeta3", C.c_double), ("zeta4", C.c_double),
        ("forchheimer", C.c_int32),
        ("T_init", C.c_double),
        ("ext_accel", C.c_double * 2),
        ("tau_v", C.c_double), ("tau_T", C.c_double),
        ("gbeta", C.c_double),
        ("Ra_I", C.c_double), ("Qv", C.c_double),
        ("dtype", C.c_int32),
        ("checkpoint_every", C.c_int32),
        ("layout", C.c_int32),
        ("steps_per_launch", C.c_int32),
    ]


class LbmObs(C.Structure):
    _fields_ = [
        ("nu_hot", C.c_double), ("nu_cold", C.c_double), ("max_speed", C.c_double),
        ("mass_err", C.c_double), ("step", C.c_int64), ("diverged", C.c_int32),
        ("why", C.c_int32), ("T_min", C.c_double), ("T_max", C.c_double),
        ("phip_dev", C.c_double),
    ]


class LbmError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}: {detail}")


_lib = None


def library() -> C.CDLL:
    """Load liblbmpm.so; raises when it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1308_2071_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, sz, i64, i32, dbl = C.c_void_p, C.c_size_t, C.c_int64, C.c_int32, C.c_double
    P = C.POINTER(LbmParams)
    sig = {
        "lbm_default_params": [P],
        "lbm_derived": [P, C.POINTER(C.c_double)],
        "lbm_workspace_size": [P, i64, C.POINTER(sz)],
        "lbm_init": [C.POINTER(vp), P, vp, vp, dbl, vp, sz, vp],
        "lbm_step": [vp, i64],
        "lbm_observables": [vp, C.POINTER(LbmObs), vp, vp, vp, vp],
        "lbm_grad": [vp, dbl, vp, vp],
        "lbm_stream_function": [vp, vp],
        "lbm_state_size": [vp, C.POINTER(sz)],
        "lbm_save": [vp, vp, sz],
        "lbm_load": [vp, vp, sz],
        "lbm_destroy": [vp],
        "lbm_batch_workspace_size": [i32, P, C.POINTER(sz)],
        "lbm_batch_init": [C.POINTER(vp), i32, P, C.POINTER(C.c_double), vp, sz, vp, C.c_char_p],
        "lbm_batch_step": [vp, i64],
        "lbm_batch_observables": [vp, C.POINTER(LbmObs)],
        "lbm_batch_fields": [vp, i32, vp, vp, vp, vp],
        "lbm_batch_shape": [vp, C.POINTER(i32)],
        "lbm_step_shape": [vp, C.POINTER(i32)],
        "lbm_run_noalloc": [P, vp, vp, dbl, i64, C.POINTER(LbmObs), vp, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int32
    L.lbm_status_string.argtypes = [C.c_int32]
    L.lbm_status_string.restype = C.c_char_p
    L.lbm_last_error.argtypes = []
    L.lbm_last_error.restype = C.c_char_p
    _lib = L
    return L


EXPORTED = (
    "lbm_default_params", "lbm_derived", "lbm_workspace_size", "lbm_init", "lbm_step",
    "lbm_observables", "lbm_grad", "lbm_stream_function", "lbm_state_size", "lbm_save", "lbm_load", "lbm_destroy",
    "lbm_batch_workspace_size", "lbm_batch_init", "lbm_batch_step", "lbm_batch_observables",
    "lbm_batch_fields", "lbm_batch_shape", "lbm_step_shape", "lbm_status_string",
    "lbm_last_error", "lbm_run_noalloc",
)


def status_string(s: int) -> str:
    return library().lbm_status_string(int(s)).decode()


def last_error() -> str:
    return library().lbm_last_error().decode()


def check(status: int, where: str) -> int:
    if status != LBM_OK:
        raise LbmError(status, where, last_error())
    return status


def ptr(t) -> int | None:
    """Device pointer of a torch tensor (None passes NULL)."""
    if t is None:
        return None
    return t.data_ptr()


def current_stream_handle(device=None) -> int | None:
    import torch
    return torch.cuda.current_stream(device).cuda_stream or None
