"""Gradient of the strain-squared loss through the D3Q19 MRT run, as a torch.autograd.Function.

    J(u0, F) = sum_x S(x, N) : S(x, N)

S is the Yu strain (which equals the Chai strain, Section 5.1 of the paper) of the
pre-collision state after N steps started from g^0 = g^eq(0, rho0 u0), with the body-force
field F (Guo forcing), at the rate the viscosity model gives it (constant, lagged
Smagorinsky or power law, implicit Smagorinsky). ``backward`` runs the hand-written adjoint
kernels of the library: the forward sweep stores the state (populations and, for the lagged
models, the s_nu field) every ``every`` steps; the reverse sweep reloads each checkpoint,
recomputes its segment saving the per-step adjoint record (3 floats per node for a constant
viscosity: j; 10 for a strain-dependent one), then runs the adjoint steps backwards through
the segment in one lbm_adjoint_steps call; lbm_init_adjoint maps the last adjoint state onto
u0. Peak extra memory: ceil(N/every) states plus ``every`` records.

With ``record_all`` the forward sweep keeps every step's record instead (N records: 12 bytes
per node and step for a constant viscosity, 40 for a strain-dependent one; 12.6 GB and
42 GB for 500 steps at 128^3, well inside one GPU's HBM), and the reverse sweep is the
adjoint steps alone, with no recompute. Both modes give the same bits: the recompute
reproduces the forward's records exactly.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import torch

from . import capi
from .lbm import LBM


@dataclass
class StrainLossProblem:
    params: capi.Params   # D3Q19, any viscosity kind; force / force_field are set per call
    nsteps: int
    every: int = 50
    record_all: bool = False  # keep every step's adjoint record from the forward sweep


class StrainLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0: torch.Tensor, F: torch.Tensor, prob: StrainLossProblem):
        p0 = prob.params
        N = p0.N
        shape = (p0.nz, p0.ny, p0.nx)
        Ff = F.detach().to(torch.float32).reshape(3, N).contiguous()
        params = replace(p0, force=(0.0, 0.0, 0.0), force_field=Ff)
        rho_u = torch.cat([torch.zeros(1, N, device=u0.device, dtype=torch.float32),
                           u0.detach().to(torch.float32).reshape(3, N)], dim=0).contiguous()
        sim = LBM(params, rho_u)
        checkpoints, rec = [], None
        if prob.record_all:
            rec = torch.empty((prob.nsteps, sim.save_planes, N), dtype=torch.float32, device=u0.device)
            if prob.nsteps:
                sim.step(prob.nsteps, save=rec)
        else:
            for n0 in range(0, prob.nsteps, prob.every):
                checkpoints.append(sim.save_state())
                sim.step(min(prob.every, prob.nsteps - n0))
        lam = torch.empty((sim.adjoint_planes, N), dtype=torch.float32, device=u0.device)
        gF = torch.zeros((3, N), dtype=torch.float32, device=u0.device)
        J = capi.lbm_strain_loss_seed(sim.ctx, lam, gF)
        ctx.sim, ctx.checkpoints, ctx.rec, ctx.lam, ctx.gF, ctx.rho_u, ctx.Ff = sim, checkpoints, rec, lam, gF, rho_u, Ff
        ctx.prob, ctx.shape = prob, shape
        return torch.tensor(J, dtype=torch.float64, device=u0.device)

    @staticmethod
    def backward(ctx, gJ):
        sim, prob, N = ctx.sim, ctx.prob, ctx.prob.params.N
        lam, gF = ctx.lam, ctx.gF
        lam2 = torch.empty_like(lam)
        if prob.record_all:
            if prob.nsteps:
                capi.lbm_adjoint_steps(sim.ctx, prob.nsteps, ctx.rec, lam, lam2, gF)
            ctx.rec = None
        else:
            rec = torch.empty((prob.every, sim.save_planes, N), dtype=torch.float32, device=lam.device)
            for seg in reversed(range(len(ctx.checkpoints))):
                n0 = seg * prob.every
                k = min(prob.every, prob.nsteps - n0)
                sim.load_state(ctx.checkpoints[seg])
                sim.step(k, save=rec)
                capi.lbm_adjoint_steps(sim.ctx, k, rec, lam, lam2, gF)
        gu = torch.empty((3, N), dtype=torch.float32, device=lam.device)
        capi.lbm_init_adjoint(sim.ctx, ctx.rho_u, lam, gu)
        scale = gJ.to(torch.float32)
        grad_u0 = (gu * scale).reshape((3,) + ctx.shape)
        grad_F = (gF * scale).reshape((3,) + ctx.shape)
        sim.close()
        ctx.sim = None
        return grad_u0, grad_F, None


def strain_loss(u0: torch.Tensor, F: torch.Tensor, prob: StrainLossProblem) -> torch.Tensor:
    """J(u0, F) with gradients through the library's adjoint kernels."""
    return StrainLoss.apply(u0, F, prob)
