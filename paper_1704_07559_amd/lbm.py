"""Convenience wrapper over the C ABI: owns the device buffers (torch allocations) of one
context and returns torch tensors shaped (components, nz, ny, nx). Marshalling only; every
step runs in the HIP kernels behind ``capi``."""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import capi
from .capi import Params


def device_field(a, device="cuda") -> torch.Tensor:
    """Host array (components, nz, ny, nx) -> contiguous float32 device tensor."""
    t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32))
    return t.to(device).contiguous()


def rho_u_field(drho, u, device="cuda") -> torch.Tensor:
    """(delta_rho (nz,ny,nx), u (3,nz,ny,nx)) -> the 4*N float32 layout lbm_init expects."""
    u = np.asarray(u)
    if u.shape[0] == 2:
        u = np.concatenate([u, np.zeros_like(u[:1])], axis=0)
    return device_field(np.concatenate([np.asarray(drho)[None], u], axis=0), device)


def grad_field(grad_u, device="cuda") -> torch.Tensor:
    """grad_u (3, 3, nz, ny, nx) with [a, b] = d u_b / d x_a -> the 9*N layout."""
    g = np.asarray(grad_u)
    return device_field(g.reshape((9,) + g.shape[2:]), device)


class LBM:
    def __init__(self, params: Params, rho_u: Optional[torch.Tensor] = None, grad_u: Optional[torch.Tensor] = None,
                 device: str = "cuda"):
        self.params = params
        self.device = torch.device(device)
        nbytes = capi.lbm_population_bytes(params)
        if nbytes == 0:
            raise ValueError("invalid parameters")
        self.f_a = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.f_b = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.s_nu = (torch.empty(params.N, dtype=torch.float32, device=self.device)
                     if params.visc_kind in (capi.LBM_VISC_SMAGORINSKY, capi.LBM_VISC_POWERLAW) else None)
        self._force_ref = params.force_field
        self.ctx = capi.lbm_init(params, self.f_a, self.f_b, self.s_nu, rho_u, grad_u)

    @property
    def shape(self):
        p = self.params
        return (p.nz, p.ny, p.nx)

    @property
    def ncomp(self) -> int:
        return 3 if self.params.lattice == capi.LBM_D2Q9 else 6

    def step(self, nsteps: int = 1, S_out: Optional[torch.Tensor] = None, strain_kind: int = capi.LBM_STRAIN_YU,
             save: Optional[torch.Tensor] = None):
        """Advance nsteps; ``save`` (nsteps x save_planes x N floats) receives the adjoint record."""
        capi.lbm_step(self.ctx, nsteps, S_out, strain_kind, save)

    @property
    def save_planes(self) -> int:
        return capi.lbm_save_planes(self.ctx)

    @property
    def adjoint_planes(self) -> int:
        return capi.lbm_adjoint_planes(self.ctx)

    def strain(self, kind: int = capi.LBM_STRAIN_YU) -> torch.Tensor:
        S = torch.empty((self.ncomp,) + self.shape, dtype=torch.float32, device=self.device)
        capi.lbm_strain(self.ctx, kind, S)
        return S

    def populations(self) -> torch.Tensor:
        f = torch.empty((self.params.q,) + self.shape, dtype=torch.float32, device=self.device)
        capi.lbm_get_populations(self.ctx, f)
        return f

    def set_populations(self, f: torch.Tensor):
        f = f.to(self.device, torch.float32).contiguous()
        capi.lbm_set_populations(self.ctx, f)
        torch.cuda.current_stream().synchronize()

    def reduce(self, allow_nonfinite: bool = False) -> dict:
        return self.diagnostics(capi.lbm_reduce(self.ctx, allow_nonfinite=allow_nonfinite))

    def reduce_async(self, out: torch.Tensor) -> torch.Tensor:
        """Queue the diagnostics into ``out`` (8 float64, on the device or pinned host memory)
        without waiting; ``diagnostics(out)`` reads them once the stream has passed."""
        capi.lbm_reduce_async(self.ctx, out)
        return out

    @staticmethod
    def diagnostics(v) -> dict:
        v = [float(a) for a in v]
        return {"mass": v[0], "mom": np.array(v[1:4]), "ke": v[4], "ss": v[5], "umax": v[6], "nonfinite": int(v[7])}

    def save_state(self) -> torch.Tensor:
        t = torch.empty(capi.lbm_state_bytes(self.ctx), dtype=torch.uint8, device=self.device)
        capi.lbm_save_state(self.ctx, t)
        return t

    def load_state(self, t: torch.Tensor):
        capi.lbm_load_state(self.ctx, t)

    @property
    def step_count(self) -> int:
        return capi.lbm_step_count(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            torch.cuda.current_stream().synchronize()
            capi.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
