"""A third opinion on the oracle's discrete adjoint: torch.autograd through an independent
FP64 forward written with torch CPU operations.

The forward here is written separately from oracle/d3q19.py, from the same definitions: the
equilibrium in its delta-rho form, m^eq = T g^eq, the Guo source as the derivative of g^eq
along F, the strain by the Chai contraction with a per-node rate field, the viscosity models,
pull streaming by torch.roll with halfway bounce-back, and J = sum S:S of the final state.
Only the lattice tables (c, w, T) are shared. Autograd then differentiates it with no
hand-written derivative, and J, dJ/du0 and dJ/dF must match oracle.adjoint.gradient to FP64
resolution. The cases cover constant viscosity with walls and a force field, lagged
Smagorinsky, the clamped power law with walls, and the implicit Smagorinsky coupling (here
autograd runs through a converged Newton solve), each also with the force-corrected strain
(the strain takes the non-equilibrium part plus half the Guo source)."""
import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as adj
from oracle import d3q19 as d

TT = torch.tensor(d.T, dtype=torch.float64)
TI = torch.tensor(d.TINV, dtype=torch.float64)
CC = torch.tensor(d.C, dtype=torch.float64)          # (3, 19)
WW = torch.tensor(d.W, dtype=torch.float64)
NU_ROWS = (9, 11, 13, 14, 15)
PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2))


def _w(x):
    return WW.reshape((19,) + (1,) * (x.dim() - 1))


def _geq(drho, j, rho0):
    u = j / rho0
    cu = torch.einsum("ai,a...->i...", CC, u)
    usq = (u * u).sum(0)
    return _w(cu) * (drho[None] + rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq[None]))


def _guo(j, F, rho0):
    u = j / rho0
    cu = torch.einsum("ai,a...->i...", CC, u)
    cF = torch.einsum("ai,a...->i...", CC, F)
    return _w(cu) * (3.0 * cF + 9.0 * cu * cF - 3.0 * (u * F).sum(0)[None])


def _rates(s, snu):
    """(19, ...) rate field: the base rates with the s_nu rows set to snu (a field)."""
    rows = [snu if k in NU_ROWS else torch.full_like(snu, float(s[k])) for k in range(19)]
    return torch.stack(rows)


def _strain(fneq, rates, rho0):
    M = torch.einsum("ik,k...->i...", TI, rates * torch.einsum("ki,i...->k...", TT, fneq))
    return torch.stack([-1.5 / rho0 * (CC[a] * CC[b] * M.movedim(0, -1)).sum(-1) for a, b in PAIRS])


def _ss(S):
    return S[0] ** 2 + S[1] ** 2 + S[2] ** 2 + 2.0 * (S[3] ** 2 + S[4] ** 2 + S[5] ** 2)


def _nu(S, p):
    gamma = torch.sqrt(2.0 * _ss(S))
    if p.visc_kind == "smagorinsky":
        return p.nu0 + p.c_smag ** 2 * gamma
    return torch.clamp(p.K_pl * gamma ** (p.n_pl - 1.0), p.nu_min, p.nu_max)


def _implicit(fneq, p):
    """s solving s (3 (nu0 + C^2 |P + s A|) + 1/2) = 1, with S(s) = P + s A."""
    zero = torch.zeros(fneq.shape[1:], dtype=torch.float64)
    P = _strain(fneq, _rates(p.s, zero), p.rho0)
    base = torch.zeros(19, dtype=torch.float64)
    A = _strain(fneq, _rates(base, zero + 1.0), p.rho0)
    s = torch.full_like(zero, 1.0 / (3.0 * p.nu0 + 0.5))
    for _ in range(40):
        S = P + s * A
        r = torch.sqrt(2.0 * _ss(S))
        dr = 2.0 * (P[:3] * A[:3]).sum(0) + 4.0 * (P[3:] * A[3:]).sum(0) + s * (2.0 * (A[:3] ** 2).sum(0)
                                                                             + 4.0 * (A[3:] ** 2).sum(0))
        f = s * (3.0 * (p.nu0 + p.c_smag ** 2 * r) + 0.5) - 1.0
        df = 3.0 * (p.nu0 + p.c_smag ** 2 * r) + 0.5 + s * 3.0 * p.c_smag ** 2 * dr / r
        s = s - f / df
    return s


def _stream(gp, walls):
    out = []
    ny = gp.shape[2]
    for i in range(19):
        cx, cy, cz = (int(v) for v in d.C[:, i])
        g = torch.roll(gp[i], shifts=(cz, cy, cx), dims=(0, 1, 2))
        if walls and cy != 0:
            y = torch.arange(ny).reshape(1, ny, 1)
            edge = (y == 0) if cy == 1 else (y == ny - 1)
            g = torch.where(edge, gp[d.OPP[i]], g)
        out.append(g)
    return torch.stack(out)


def torch_loss(u0, F, p, nsteps):
    shape = u0.shape[1:]
    g = _geq(torch.zeros(shape, dtype=torch.float64), p.rho0 * u0, p.rho0)
    snu = torch.full(shape, float(p.s[9]), dtype=torch.float64)

    def state(g):
        drho = g.sum(0)
        j = torch.einsum("ai,i...->a...", CC, g) + 0.5 * F
        geq = _geq(drho, j, p.rho0)
        fneq = g - geq
        # what the strain takes: with the correction, plus half the Guo source
        fs = fneq + 0.5 * _guo(j, F, p.rho0) if p.force_corrected else fneq
        return j, geq, fs

    for _ in range(nsteps):
        j, geq, fs = state(g)
        if p.visc_kind in ("smagorinsky", "powerlaw"):
            snu = 1.0 / (3.0 * _nu(_strain(fs, _rates(p.s, snu), p.rho0), p) + 0.5)
        elif p.visc_kind == "smagorinsky_implicit":
            snu = _implicit(fs, p)
        rates = _rates(p.s, snu)
        m = torch.einsum("ki,i...->k...", TT, g)
        meq = torch.einsum("ki,i...->k...", TT, geq)
        SF = torch.einsum("ki,i...->k...", TT, _guo(j, F, p.rho0))
        mpost = m - rates * (m - meq) + (1.0 - 0.5 * rates) * SF
        g = _stream(torch.einsum("ik,k...->i...", TI, mpost), p.walls_y)
    j, geq, fs = state(g)
    if p.visc_kind == "smagorinsky_implicit":
        snu = _implicit(fs, p)
    return _ss(_strain(fs, _rates(p.s, snu), p.rho0)).sum()


CASES = {
    "const_walls": dict(walls_y=True),
    "smagorinsky": dict(visc_kind="smagorinsky", nu0=0.01, c_smag=0.3),
    "powerlaw_walls": dict(visc_kind="powerlaw", visc_strain="chai", K_pl=0.01, n_pl=0.6, nu_min=2e-3, nu_max=0.05,
                           walls_y=True),
    "smagorinsky_implicit": dict(visc_kind="smagorinsky_implicit", nu0=0.005, c_smag=0.4),
    "const_walls_corrected": dict(walls_y=True, force_corrected=True),
    "smagorinsky_corrected": dict(visc_kind="smagorinsky", nu0=0.01, c_smag=0.3, force_corrected=True),
    "powerlaw_walls_corrected": dict(visc_kind="powerlaw", visc_strain="chai", K_pl=0.01, n_pl=0.6, nu_min=2e-3,
                                     nu_max=0.05, walls_y=True, force_corrected=True),
    "smagorinsky_implicit_corrected": dict(visc_kind="smagorinsky_implicit", nu0=0.005, c_smag=0.4,
                                           force_corrected=True),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_adjoint_matches_autograd(case):
    shape, nsteps = (4, 5, 6), 6
    u0 = synth.random_vector(shape, seed=61, scale=0.03)
    F = synth.uniform_random_force(shape, seed=62, amp=1e-3)
    p = d.Params(s=d.default_rates(0.7), **CASES[case])
    J, gu, gF = adj.gradient(u0, F, p, nsteps, every=4)
    ut = torch.tensor(u0, requires_grad=True)
    Ft = torch.tensor(F, requires_grad=True)
    Jt = torch_loss(ut, Ft, p, nsteps)
    Jt.backward()
    assert abs(Jt.item() - J) <= 1e-12 * J
    assert np.abs(ut.grad.numpy() - gu).max() <= 1e-9 * np.abs(gu).max()
    assert np.abs(Ft.grad.numpy() - gF).max() <= 1e-9 * np.abs(gF).max()
    if case.startswith("powerlaw_walls"):
        # both branches occur in the last steps: nodes on the nu_max clamp (zero slope) and
        # nodes on the power law itself
        sim = d.Simulation(adj._with_force(p, F), d.init_populations(np.zeros(shape), u0, adj._with_force(p, F)))
        sim.step(nsteps)
        nu = (1.0 / sim.s_nu - 0.5) / 3.0
        clamped = np.isclose(nu, p.nu_max, rtol=1e-12)
        assert 0 < clamped.sum() < clamped.size
