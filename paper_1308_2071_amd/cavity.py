"""Torch-facing conveniences over the ABI: a cavity with a torch-owned workspace, a batch of
cavities, and the adjoint as a ``torch.autograd.Function``."""
from __future__ import annotations

import numpy as np
import torch

from . import (LBM_FP64, lbm_batch_fields, lbm_batch_init, lbm_batch_observables,
               lbm_batch_shape,
               lbm_batch_step, lbm_batch_workspace_size, lbm_destroy, lbm_grad, lbm_init,
               lbm_load, lbm_observables, lbm_save, lbm_state_size, lbm_step, lbm_stream_function,
               lbm_workspace_size,
               make_params)
from ._abi import LBM_OK, LbmParams


def _torch_dtype(p: LbmParams):
    return torch.float64 if p.dtype == LBM_FP64 else torch.float32


def _obs_dict(o, status=LBM_OK) -> dict:
    return dict(nu_hot=o.nu_hot, nu_cold=o.nu_cold, max_speed=o.max_speed, mass_err=o.mass_err,
                step=o.step, diverged=bool(o.diverged), why=int(o.why), T_min=o.T_min,
                T_max=o.T_max, phip_dev=o.phip_dev, status=status)


class Cavity:
    """One cavity on one GPU.  ``params`` is an LbmParams or a dict of its fields; phi and K are
    [ny][nx] tensors (any device/dtype; copied) or None for uniform values."""

    def __init__(self, params, phi=None, K=None, phi_uniform: float = 1.0,
                 nsteps_max: int = 0, device="cuda"):
        self.p = params if isinstance(params, LbmParams) else make_params(**params)
        self.device = torch.device(device)
        self.dtype = _torch_dtype(self.p)
        self.nx, self.ny = self.p.nx, self.p.ny
        nbytes = lbm_workspace_size(self.p, nsteps_max)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        cv = lambda t: None if t is None else t.to(self.device, self.dtype).contiguous()
        phi_d, K_d = cv(phi), cv(K)
        self.ctx = lbm_init(self.p, phi_d, K_d, phi_uniform, self.workspace)
        del phi_d, K_d

    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        lbm_step(self.ctx, n)
        return self

    def observables(self, fields: bool = True) -> dict:
        """Nu_hot, Nu_cold (Eq. (38)), max |u|, mass deviation, step, min and max T,
        max |phi p - rho0 cs^2|, the divergence flag and its reasons (LBM_DIV_* bits); with
        ``fields`` also u_x, u_y, the dynamic pressure p - rho0 cs^2 / phi and T as [ny][nx]
        tensors of the cavity's dtype."""
        if fields:
            ux, uy, p, T = (torch.empty(self.ny, self.nx, dtype=self.dtype, device=self.device)
                            for _ in range(4))
        else:
            ux = uy = p = T = None
        s, o = lbm_observables(self.ctx, ux, uy, p, T)
        d = _obs_dict(o, s)
        if fields:
            d.update(ux=ux, uy=uy, p=p, T=T)
        return d

    def stream_function(self):
        psi = torch.empty(self.ny, self.nx, dtype=self.dtype, device=self.device)
        lbm_stream_function(self.ctx, psi)
        return psi

    def grad(self, dJ: float = 1.0):
        gphi = torch.empty(self.ny, self.nx, dtype=torch.float64, device=self.device)
        gK = torch.empty(self.ny, self.nx, dtype=torch.float64, device=self.device)
        lbm_grad(self.ctx, dJ, gphi, gK)
        return gphi, gK

    def save(self) -> np.ndarray:
        buf = np.empty(lbm_state_size(self.ctx), dtype=np.uint8)
        lbm_save(self.ctx, buf)
        return buf

    def load(self, buf: np.ndarray):
        lbm_load(self.ctx, np.ascontiguousarray(buf))


class Batch:
    """Many independent cavities stepped together (uniform phi and K = Da L^2 per cavity)."""

    def __init__(self, params_list, phi_uniform, device="cuda", tune_cache_path=None):
        self.params = [p if isinstance(p, LbmParams) else make_params(**p) for p in params_list]
        self.n = len(self.params)
        self.device = torch.device(device)
        nbytes = lbm_batch_workspace_size(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ctx = lbm_batch_init(self.params, list(phi_uniform), self.workspace,
                                  tune_cache_path=tune_cache_path)

    def step(self, n: int = 1):
        lbm_batch_step(self.ctx, n)
        return self

    def observables(self):
        s, obs = lbm_batch_observables(self.ctx, self.n)
        return s, [_obs_dict(o) for o in obs]

    def fields(self, i: int) -> dict:
        p = self.params[i]
        dt = _torch_dtype(p)
        ux, uy, pr, T = (torch.empty(p.ny, p.nx, dtype=dt, device=self.device) for _ in range(4))
        lbm_batch_fields(self.ctx, i, ux, uy, pr, T)
        return dict(ux=ux, uy=uy, p=pr, T=T)

    def shape(self):
        return lbm_batch_shape(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NuHot(torch.autograd.Function):
    """J = hot-wall average Nusselt number (Eq. (38)) after ``nsteps`` steps from rest, as a
    function of the per-node porosity phi and permeability K.  Forward runs the HIP time step
    with a checkpoint every ``checkpoint_every`` steps; backward runs the HIP discrete adjoint
    (checkpoint-and-recompute).  Gradients come back in phi's dtype."""

    @staticmethod
    def forward(ctx, phi, K, params: dict, nsteps: int, checkpoint_every: int = 100):
        p = dict(params)
        p["checkpoint_every"] = int(checkpoint_every)
        cav = Cavity(p, phi=phi.detach(), K=K.detach(), nsteps_max=nsteps, device=phi.device)
        cav.step(nsteps)
        o = cav.observables(fields=False)
        ctx.cav = cav
        ctx.dtypes = (phi.dtype, K.dtype)
        return torch.tensor(o["nu_hot"], dtype=phi.dtype, device=phi.device)

    @staticmethod
    def backward(ctx, gJ):
        gphi, gK = ctx.cav.grad(float(gJ))   # repeatable: the tape stays until ctx is freed
        return gphi.to(ctx.dtypes[0]), gK.to(ctx.dtypes[1]), None, None, None
