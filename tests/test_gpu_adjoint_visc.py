"""Parity of the adjoint kernels for a strain-dependent viscosity (lagged Smagorinsky, lagged
power law, implicit Smagorinsky) with the FP64 oracle of oracle/adjoint_visc.py, through the
C ABI and through the checkpointed torch.autograd.Function.

Tolerances as for the constant-viscosity adjoint: one kernel call max|d| / max|ref| <= 1e-5
(FP32 against FP64), whole gradients over tens of steps <= 1e-4.
"""
import numpy as np
import pytest

import synth
from oracle import adjoint as adj
from oracle import adjoint_visc as av
from oracle import d3q19 as od
from tests._common import needs_gpu, spec_params, to_np

pytestmark = [pytest.mark.gpu, needs_gpu]

MODELS = {
    "smag_yu": dict(visc="smagorinsky", drive="yu", nu0=0.01, c_smag=0.4),
    "smag_chai": dict(visc="smagorinsky", drive="chai", nu0=0.002, c_smag=0.3),
    "powerlaw_thinning": dict(visc="powerlaw", drive="chai", K_pl=0.02, n_pl=0.5, nu_min=1e-3, nu_max=0.5),
    "powerlaw_thickening": dict(visc="powerlaw", drive="yu", K_pl=2.0, n_pl=1.5, nu_min=1e-3, nu_max=1.0),
    "implicit_yu": dict(visc="smagorinsky_implicit", drive="yu", nu0=0.01, c_smag=0.4),
    "implicit_chai": dict(visc="smagorinsky_implicit", drive="chai", nu0=0.002, c_smag=0.3),
}


def _rel(a, b):
    return float(np.abs(np.asarray(a, dtype=np.float64) - b).max() / np.abs(b).max())


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _state(shape, seed, p):
    u = synth.random_vector(shape, seed=seed, scale=0.05)
    return _f32(od.init_populations(np.zeros(shape), u, p) + synth.random_state(19, shape, seed=seed + 1, scale=3e-3))


def _s_field(shape, seed):
    return _f32(1.0 / (3.0 * (0.02 + 0.01 * synth.random_state(1, shape, seed=seed, scale=1.0)[0] ** 2) + 0.5))


def _setup(name, shape, walls, seed):
    import torch
    from paper_1704_07559_amd import lbm
    F = _f32(synth.uniform_random_force(shape, seed=seed, amp=1e-4))
    op, cp, _ = spec_params(shape, tau=0.8, walls=walls, force=F, **MODELS[name])
    g = _state(shape, seed + 1, op)
    sim = lbm.LBM(cp)
    sim.set_populations(torch.as_tensor(g.astype(np.float32)).cuda())
    sp = None
    if sim.s_nu is not None:
        sp = _s_field(shape, seed + 2)
        sim.s_nu.copy_(torch.as_tensor(sp.reshape(-1).astype(np.float32)))
    return op, cp, F, g, sp, sim


@pytest.mark.parametrize("shape", [(5, 9, 70), (3, 8, 64)])
@pytest.mark.parametrize("name,walls", [("smag_yu", False), ("smag_chai", True), ("powerlaw_thinning", True),
                                        ("powerlaw_thickening", False), ("implicit_yu", True),
                                        ("implicit_chai", False)])
def test_adjoint_step_matches_oracle(name, walls, shape):
    import torch
    from paper_1704_07559_amd import capi
    op, cp, F, g, sp, sim = _setup(name, shape, walls, 30)
    N = cp.N
    assert sim.save_planes == 10
    A = sim.adjoint_planes
    assert A == (20 if sp is not None else 19)
    rec = torch.empty((1, 10, N), device="cuda")
    sim.step(1, save=rec)
    lam_in = _f32(synth.random_state(A, shape, seed=40, scale=1.0))
    lam_t = torch.as_tensor(lam_in.astype(np.float32)).cuda().reshape(A, N).contiguous()
    lam_out = torch.empty_like(lam_t)
    gF = torch.zeros((3, N), device="cuda")
    capi.lbm_adjoint_step(sim.ctx, rec[0], lam_t, lam_out, gF)
    ref_lam, ref_lams, ref_gF = av.adjoint_step_visc(lam_in[:19], lam_in[19] if sp is not None else None, g, sp, F,
                                                     adj._with_force(op, F))
    out = to_np(lam_out).reshape((A,) + shape)
    assert _rel(out[:19], ref_lam) < 1e-5
    assert _rel(to_np(gF).reshape(ref_gF.shape), ref_gF) < 1e-5
    if sp is not None:
        assert _rel(out[19], ref_lams) < 1e-5
    sim.close()


@pytest.mark.parametrize("name", sorted(MODELS))
def test_loss_seed_matches_oracle(name):
    import torch
    from paper_1704_07559_amd import capi
    shape = (4, 11, 67)
    op, cp, F, g, sp, sim = _setup(name, shape, False, 50)
    N = cp.N
    A = sim.adjoint_planes
    lam = torch.empty((A, N), device="cuda")
    gF = torch.zeros((3, N), device="cuda")
    J = capi.lbm_strain_loss_seed(sim.ctx, lam, gF)
    Jr, lamr, lamsr, gFr = av.strain_loss_seed_visc(g, sp, F, adj._with_force(op, F))
    assert abs(J - Jr) < 1e-5 * Jr
    out = to_np(lam).reshape((A,) + shape)
    assert _rel(out[:19], lamr) < 1e-5
    assert _rel(to_np(gF).reshape(gFr.shape), gFr) < 1e-5
    if sp is not None:
        assert _rel(out[19], lamsr) < 1e-5
    sim.close()


@pytest.mark.parametrize("name,walls", [("smag_yu", False), ("powerlaw_thinning", True), ("implicit_chai", False)])
def test_strain_loss_gradient_matches_oracle(name, walls):
    """Checkpointed GPU gradient (30 steps, every 7) against the FP64 oracle gradient on
    12 x 13 x 16 nodes, u0 with u_rms 0.04 and a random force field."""
    import torch
    from paper_1704_07559_amd import autograd as ag
    shape = (12, 13, 16)
    u0 = _f32(synth.spectrum_velocity(shape, seed=1704, u_rms=0.04))
    F = _f32(synth.uniform_random_force(shape, seed=7559, amp=1e-5))
    op, cp, _ = spec_params(shape, tau=0.8, walls=walls, **MODELS[name])
    nsteps, every = 30, 7
    Jr, gur, gFr = adj.gradient(u0, F, op, nsteps, every=every)
    u0_t = torch.as_tensor(u0.astype(np.float32)).cuda().requires_grad_(True)
    F_t = torch.as_tensor(F.astype(np.float32)).cuda().requires_grad_(True)
    J = ag.strain_loss(u0_t, F_t, ag.StrainLossProblem(cp, nsteps, every))
    J.backward()
    assert abs(J.item() - Jr) < 1e-4 * Jr
    assert _rel(to_np(u0_t.grad), gur) < 1e-4
    assert _rel(to_np(F_t.grad), gFr) < 1e-4


def test_record_planes_and_validation():
    """Constant viscosity keeps the 3-plane record and 19 adjoint planes; D2Q9 has none."""
    from paper_1704_07559_amd import capi, lbm
    _, cp, _ = spec_params((2, 3, 64), tau=0.8)
    sim = lbm.LBM(cp)
    assert (sim.save_planes, sim.adjoint_planes) == (3, 19)
    sim.close()
    p2 = capi.Params(nx=16, ny=8, nz=1, lattice=capi.LBM_D2Q9, s=[0.0, 1.19, 1.4, 0.0, 1.2, 0.0, 1.2, 1.25, 1.25])
    sim2 = lbm.LBM(p2)
    assert (sim2.save_planes, sim2.adjoint_planes) == (0, 0)
    sim2.close()


# (model, nsteps, (nz, ny, nx), walls): whole rows with masked lanes (ny not a multiple of the
# block's rows, or nx not a power of two), whole rows through LDS, part rows (nx = 512), with
# and without y-walls; nsteps 1 and 2 have no intermediate (row-interleaved) state or one.
SWEEPS = [("const", 5, (4, 9, 64), False), ("const", 4, (4, 8, 64), False), ("const", 1, (4, 8, 64), True),
          ("smag_yu", 3, (4, 9, 64), False), ("smag_yu", 3, (2, 4, 512), True), ("smag_chai", 2, (4, 8, 64), True),
          ("implicit_chai", 6, (4, 9, 64), False), ("implicit_yu", 4, (4, 8, 64), True),
          ("powerlaw_thinning", 5, (3, 5, 96), False)]


@pytest.mark.parametrize("name,nsteps,shape,walls", SWEEPS)
def test_adjoint_steps_equals_single_steps(name, nsteps, shape, walls):
    """lbm_adjoint_steps (one call, lambda ping-pong inside the library, the intermediate
    states row-interleaved) is bit-identical to nsteps lbm_adjoint_step calls on canonical
    planes, for odd and even nsteps and every launch shape; the result lands in lam_a."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    F = _f32(synth.uniform_random_force(shape, seed=60, amp=1e-4))
    kw = {} if name == "const" else MODELS[name]
    op, cp, _ = spec_params(shape, tau=0.8, walls=walls, force=F, **kw)
    u = synth.random_vector(shape, seed=61, scale=0.05)
    sim = lbm.LBM(cp, lbm.rho_u_field(np.zeros(shape), u))
    N, R, A = cp.N, sim.save_planes, sim.adjoint_planes
    rec = torch.empty((nsteps, R, N), device="cuda")
    sim.step(nsteps, save=rec)
    lam0 = torch.as_tensor(synth.random_state(A, shape, seed=62, scale=1.0).astype(np.float32)).cuda().reshape(A, N)
    a, b, gF = lam0.clone(), torch.empty_like(lam0), torch.zeros((3, N), device="cuda")
    capi.lbm_adjoint_steps(sim.ctx, nsteps, rec, a, b, gF)
    x, y, gF1 = lam0.clone(), torch.empty_like(lam0), torch.zeros((3, N), device="cuda")
    for n in reversed(range(nsteps)):
        capi.lbm_adjoint_step(sim.ctx, rec[n], x, y, gF1)
        x, y = y, x
    assert torch.equal(a, x) and torch.equal(gF, gF1)
    sim.close()
