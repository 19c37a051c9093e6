"""MI355X (gfx950) implementation of the coupled D2Q9 / D2Q5 multiple-relaxation-time lattice
Boltzmann model for convection heat transfer in porous media at the REV scale (Liu, He, Li,
Tao, arXiv:1308.2071).

The compute path is the HIP library ``liblbmpm.so`` behind the C ABI of ``include/lbm.h``.  This
package is its Python binding: functions with the ABI's names (argument marshalling only) and two
conveniences built from them, :class:`Cavity` (one cavity with a torch-owned workspace) and
:class:`NuHot` (a ``torch.autograd.Function`` whose backward is the library's discrete adjoint).
"""
from __future__ import annotations

import ctypes as C

from . import _abi
from ._abi import (LBM_DIV_NONFINITE, LBM_DIV_SPEED, LBM_DIV_TEMPERATURE,
                   LBM_FP32, LBM_FP32_F64, LBM_FP64, LBM_LAYOUT_AA, LBM_LAYOUT_PULL,
                   LBM_PERIODIC, LBM_WALL_ADIABATIC, LBM_WALL_ISOTHERMAL, LbmError, LbmObs,
                   LbmParams, check, library, ptr)

__all__ = [
    "LbmParams", "LbmObs", "LbmError", "LBM_FP32", "LBM_FP64", "LBM_FP32_F64",
    "LBM_LAYOUT_PULL", "LBM_LAYOUT_AA",
    "LBM_WALL_ISOTHERMAL",
    "LBM_WALL_ADIABATIC", "LBM_PERIODIC", "LBM_DIV_NONFINITE", "LBM_DIV_SPEED",
    "LBM_DIV_TEMPERATURE", "library", "make_params", "params_dict",
    "lbm_default_params", "lbm_derived", "lbm_workspace_size", "lbm_init", "lbm_step",
    "lbm_observables", "lbm_grad", "lbm_stream_function", "lbm_state_size", "lbm_save", "lbm_load", "lbm_destroy",
    "lbm_batch_workspace_size", "lbm_batch_init", "lbm_batch_step", "lbm_batch_observables",
    "lbm_batch_fields", "lbm_batch_shape", "lbm_step_shape", "lbm_status_string",
    "lbm_last_error", "lbm_run_noalloc", "Cavity", "Batch", "NuHot",
]

_ARRAY_FIELDS = ("bc", "T_wall", "ext_accel")


# ---- the ABI, one function per entry point --------------------------------------------------

def lbm_default_params() -> LbmParams:
    p = LbmParams()
    check(library().lbm_default_params(C.byref(p)), "lbm_default_params")
    return p


def lbm_derived(p: LbmParams) -> dict:
    out = (C.c_double * 10)()
    check(library().lbm_derived(C.byref(p), out), "lbm_derived")
    names = ("L", "tau_v", "tau_T", "nu_e", "nu", "gbeta", "dT", "T0", "K", "Q")
    return dict(zip(names, list(out)))


def lbm_workspace_size(p: LbmParams, nsteps_max: int = 0) -> int:
    n = C.c_size_t()
    check(library().lbm_workspace_size(C.byref(p), int(nsteps_max), C.byref(n)),
          "lbm_workspace_size")
    return n.value


def lbm_init(p: LbmParams, phi, K, phi_uniform: float, workspace, stream=None) -> int:
    """phi, K: device tensors [ny][nx] of the params' dtype, or None; workspace: device uint8
    tensor of at least lbm_workspace_size() bytes (kept alive by the caller)."""
    h = C.c_void_p()
    if stream is None:
        stream = _abi.current_stream_handle(workspace.device)
    check(library().lbm_init(C.byref(h), C.byref(p), ptr(phi), ptr(K), float(phi_uniform),
                             ptr(workspace), workspace.numel() * workspace.element_size(),
                             stream), "lbm_init")
    return h.value


def lbm_step(ctx: int, nsteps: int) -> None:
    check(library().lbm_step(ctx, int(nsteps)), "lbm_step")


def lbm_observables(ctx: int, ux=None, uy=None, p=None, T=None):
    """Returns (status, LbmObs); LBM_E_DIVERGED is returned, other failures raise."""
    o = LbmObs()
    s = library().lbm_observables(ctx, C.byref(o), ptr(ux), ptr(uy), ptr(p), ptr(T))
    if s not in (_abi.LBM_OK, _abi.LBM_E_DIVERGED):
        check(s, "lbm_observables")
    return s, o


def lbm_grad(ctx: int, dJ: float, dJ_dphi=None, dJ_dK=None) -> None:
    check(library().lbm_grad(ctx, float(dJ), ptr(dJ_dphi), ptr(dJ_dK)), "lbm_grad")


def lbm_stream_function(ctx: int, psi) -> None:
    check(library().lbm_stream_function(ctx, ptr(psi)), "lbm_stream_function")


def lbm_state_size(ctx: int) -> int:
    n = C.c_size_t()
    check(library().lbm_state_size(ctx, C.byref(n)), "lbm_state_size")
    return n.value


def lbm_save(ctx: int, host_buf) -> None:
    """host_buf: writable contiguous host buffer (e.g. a numpy uint8 array)."""
    addr = host_buf.ctypes.data
    check(library().lbm_save(ctx, addr, host_buf.nbytes), "lbm_save")


def lbm_load(ctx: int, host_buf) -> None:
    addr = host_buf.ctypes.data
    check(library().lbm_load(ctx, addr, host_buf.nbytes), "lbm_load")


def lbm_destroy(ctx: int) -> None:
    check(library().lbm_destroy(ctx), "lbm_destroy")


def lbm_batch_workspace_size(params) -> int:
    arr = (LbmParams * len(params))(*params)
    n = C.c_size_t()
    check(library().lbm_batch_workspace_size(len(params), arr, C.byref(n)),
          "lbm_batch_workspace_size")
    return n.value


def lbm_batch_init(params, phi_uniform, workspace, stream=None, tune_cache_path=None) -> int:
    n = len(params)
    arr = (LbmParams * n)(*params)
    phis = (C.c_double * n)(*[float(v) for v in phi_uniform])
    h = C.c_void_p()
    if stream is None:
        stream = _abi.current_stream_handle(workspace.device)
    path = tune_cache_path.encode() if tune_cache_path else None
    check(library().lbm_batch_init(C.byref(h), n, arr, phis, ptr(workspace),
                                   workspace.numel() * workspace.element_size(), stream, path),
          "lbm_batch_init")
    return h.value


def lbm_batch_step(ctx: int, nsteps: int) -> None:
    check(library().lbm_batch_step(ctx, int(nsteps)), "lbm_batch_step")


def lbm_batch_observables(ctx: int, n: int):
    o = (LbmObs * n)()
    s = library().lbm_batch_observables(ctx, o)
    if s not in (_abi.LBM_OK, _abi.LBM_E_DIVERGED):
        check(s, "lbm_batch_observables")
    return s, list(o)


def lbm_batch_fields(ctx: int, i: int, ux=None, uy=None, p=None, T=None) -> None:
    check(library().lbm_batch_fields(ctx, int(i), ptr(ux), ptr(uy), ptr(p), ptr(T)),
          "lbm_batch_fields")


def lbm_batch_shape(ctx: int):
    out = (C.c_int32 * 8)()
    check(library().lbm_batch_shape(ctx, out), "lbm_batch_shape")
    return tuple(out)


def lbm_step_shape(ctx: int):
    out = (C.c_int32 * 4)()
    check(library().lbm_step_shape(ctx, out), "lbm_step_shape")
    return tuple(out)


def lbm_run_noalloc(p: LbmParams, phi, K, phi_uniform: float, nsteps: int, ux=None, uy=None,
                    pr=None, T=None, stream=None):
    """One cavity run from rest for nsteps steps in the library's own device array (no
    workspace, nothing allocated); returns (status, LbmObs) like lbm_observables."""
    o = LbmObs()
    if stream is None:
        dev = next((t.device for t in (phi, K, ux, uy, pr, T) if t is not None), None)
        stream = _abi.current_stream_handle(dev)
    s = library().lbm_run_noalloc(C.byref(p), ptr(phi), ptr(K), float(phi_uniform),
                                  int(nsteps), C.byref(o), ptr(ux), ptr(uy), ptr(pr), ptr(T),
                                  stream)
    if s not in (_abi.LBM_OK, _abi.LBM_E_DIVERGED):
        check(s, "lbm_run_noalloc")
    return s, o


def lbm_status_string(s: int) -> str:
    return _abi.status_string(s)


def lbm_last_error() -> str:
    return _abi.last_error()


# ---- parameters from plain dicts --------------------------------------------------------------

def make_params(**kw) -> LbmParams:
    """lbm_params from keyword arguments over the paper's defaults; dtype may be 'fp32', 'fp64' or
    'fp32_f64' (FP32 storage, FP64 arithmetic); layout may be 'pull' or 'aa'."""
    p = lbm_default_params()
    for k, v in kw.items():
        if k == "dtype" and isinstance(v, str):
            v = {"fp32": LBM_FP32, "fp64": LBM_FP64, "fp32_f64": LBM_FP32_F64}[v]
        if k == "layout" and isinstance(v, str):
            v = {"pull": LBM_LAYOUT_PULL, "aa": LBM_LAYOUT_AA}[v]
        if k in _ARRAY_FIELDS:
            arr = getattr(p, k)
            for i, x in enumerate(v):
                arr[i] = x
        elif k in dict(LbmParams._fields_):
            setattr(p, k, v)
        else:
            raise KeyError(f"unknown lbm_params field {k!r}")
    return p


def params_dict(p: LbmParams) -> dict:
    d = {}
    for name, _ in LbmParams._fields_:
        v = getattr(p, name)
        d[name] = tuple(v) if name in _ARRAY_FIELDS else v
    return d


from .cavity import Batch, Cavity, NuHot  # noqa: E402
