"""Parity of the force-corrected strain (strain_force_correction = 1) with the FP64 oracle on
D3Q19, D3Q15 and D2Q9.

The force here is large (field amplitude 1e-2 against a random state of amplitude 3e-3), so
the correction changes the strain by far more than the 1e-4 parity tolerance; each case
checks that the uncorrected oracle strain is out of tolerance. The adjoint of the corrected
strain (D3Q19: step, loss seed, whole gradient) is compared with oracle/adjoint*.py run with
the correction, and each case checks that the uncorrected adjoint differs.
"""
import numpy as np
import pytest

import synth
from oracle import d2q9 as o9
from oracle import d3q15 as o15
from oracle import d3q19 as o19
from tests._common import needs_gpu, pop_rel_err, spec_params, strain_rel_err, to_np

pytestmark = [pytest.mark.gpu, needs_gpu]

SHAPES = {19: (4, 10, 69), 15: (5, 9, 70), 9: (1, 23, 131)}
ORACLE = {19: o19, 15: o15, 9: o9}


def _spec(q, shape, **kw):
    if q == 19:
        op, cp, _ = spec_params(shape, **kw)
        return op, cp
    if q == 15:
        from tests.test_gpu_d3q15 import _spec as spec15
        return spec15(shape, **kw)
    from tests.test_gpu_d2q9 import _spec as spec9
    return spec9(shape, **kw)


def _ss(S):
    w = np.array([1, 1, 1, 2, 2, 2] if S.shape[0] == 6 else [1, 1, 2], dtype=np.float64)
    return float((w.reshape((-1,) + (1,) * (S.ndim - 1)) * S * S).sum())


CASES = {
    "const_field": dict(),
    "smag_chai_walls": dict(visc="smagorinsky", drive="chai", nu0=0.01, c_smag=0.3, walls=True),
    "implicit_yu": dict(visc="smagorinsky_implicit", drive="yu", nu0=0.002, c_smag=0.3),
    "implicit_chai": dict(visc="smagorinsky_implicit", drive="chai", nu0=0.005, c_smag=0.2),
}


@pytest.mark.parametrize("q", [19, 15, 9])
@pytest.mark.parametrize("case", sorted(CASES))
def test_corrected_strain_steps(q, case):
    import torch
    from paper_1704_07559_amd import capi, lbm
    od = ORACLE[q]
    shape = SHAPES[q]
    dim = 2 if q == 9 else 3
    F = synth.uniform_random_force(shape, seed=7559, amp=1e-2)[:dim]
    op, cp = _spec(q, shape, force=F, **CASES[case])
    op.force_corrected = True
    cp.strain_force_correction = 1
    sim = lbm.LBM(cp)
    g0 = synth.random_state(q, shape, seed=11, scale=3e-3).astype(np.float32).astype(np.float64)
    sim.set_populations(torch.as_tensor(g0.astype(np.float32)).cuda())
    ref = od.Simulation(op, g0)
    plain = dict(op.__dict__)
    plain["force_corrected"] = False
    op_plain = type(op)(**plain)
    nc = 6 if dim == 3 else 3
    S = torch.empty((nc,) + shape, device="cuda")
    for n in range(3):
        S_chai = to_np(sim.strain(capi.LBM_STRAIN_CHAI))
        assert strain_rel_err(S_chai, od.strain_of_state(ref.g, op, ref.s_nu, "chai")) < 1e-4, n
        assert strain_rel_err(S_chai, od.strain_of_state(ref.g, op_plain, ref.s_nu, "chai")) > 1e-3, n
        sim.step(1, S_out=S, strain_kind=capi.LBM_STRAIN_YU)
        out = ref.step(1)
        S_yu_ref = out.S_yu if q == 19 else out[0]
        assert strain_rel_err(to_np(S), S_yu_ref) < 1e-4, n
        assert pop_rel_err(to_np(sim.populations()), ref.g, op.rho0, od.W) < 1e-5, n
    ss = _ss(od.strain_of_state(ref.g, op, ref.s_nu, "yu"))
    assert abs(sim.reduce()["ss"] - ss) < 1e-4 * ss
    sim.close()


# --- the adjoint of the force-corrected strain (D3Q19) ---------------------------------

ADJ_MODELS = {
    "const": dict(),
    "smag_yu": dict(visc="smagorinsky", drive="yu", nu0=0.01, c_smag=0.4),
    "powerlaw_thinning": dict(visc="powerlaw", drive="chai", K_pl=0.02, n_pl=0.5, nu_min=1e-3, nu_max=0.5),
    "implicit_chai": dict(visc="smagorinsky_implicit", drive="chai", nu0=0.002, c_smag=0.3),
}


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _rel(a, b):
    return float(np.abs(np.asarray(a, dtype=np.float64) - b).max() / np.abs(b).max())


def _adj_setup(name, shape, walls, seed, amp=3e-3):
    """A corrected-strain context on a random state, the force large enough that the
    correction moves every adjoint quantity well beyond the parity tolerance."""
    import torch
    from paper_1704_07559_amd import lbm
    F = _f32(synth.uniform_random_force(shape, seed=seed, amp=amp))
    op, cp, _ = spec_params(shape, tau=0.8, walls=walls, force=F, **ADJ_MODELS[name])
    op.force_corrected = True
    cp.strain_force_correction = 1
    u = synth.random_vector(shape, seed=seed + 1, scale=0.05)
    g = _f32(o19.init_populations(np.zeros(shape), u, op) + synth.random_state(19, shape, seed=seed + 2, scale=3e-3))
    sim = lbm.LBM(cp)
    sim.set_populations(torch.as_tensor(g.astype(np.float32)).cuda())
    sp = None
    if sim.s_nu is not None:
        sp = _f32(1.0 / (3.0 * (0.02 + 0.01 * synth.random_state(1, shape, seed=seed + 3, scale=1.0)[0] ** 2) + 0.5))
        sim.s_nu.copy_(torch.as_tensor(sp.reshape(-1).astype(np.float32)))
    return op, cp, F, g, sp, sim


def _uncorrected(op):
    from oracle import adjoint as adj
    q = adj._with_force(op, op.force)
    q.force_corrected = False
    return q


@pytest.mark.parametrize("name,walls", [("smag_yu", False), ("powerlaw_thinning", True), ("implicit_chai", False)])
def test_adjoint_step_with_the_correction(name, walls):
    import torch
    from oracle import adjoint as adj
    from oracle import adjoint_visc as av
    from paper_1704_07559_amd import capi
    shape = (3, 8, 64)
    op, cp, F, g, sp, sim = _adj_setup(name, shape, walls, 30)
    N = cp.N
    A = sim.adjoint_planes
    rec = torch.empty((1, 10, N), device="cuda")
    sim.step(1, save=rec)
    lam_in = _f32(synth.random_state(A, shape, seed=40, scale=1.0))
    lam_t = torch.as_tensor(lam_in.astype(np.float32)).cuda().reshape(A, N).contiguous()
    lam_out = torch.empty_like(lam_t)
    gF = torch.zeros((3, N), device="cuda")
    capi.lbm_adjoint_step(sim.ctx, rec[0], lam_t, lam_out, gF)
    sp_in = sp if sp is not None else None
    lams_in = lam_in[19] if sp is not None else None
    ref_lam, ref_lams, ref_gF = av.adjoint_step_visc(lam_in[:19], lams_in, g, sp_in, F, adj._with_force(op, F))
    out = to_np(lam_out).reshape((A,) + shape)
    assert _rel(out[:19], ref_lam) < 1e-5
    assert _rel(to_np(gF).reshape(ref_gF.shape), ref_gF) < 1e-5
    if sp is not None:
        assert _rel(out[19], ref_lams) < 1e-5
    plain = av.adjoint_step_visc(lam_in[:19], lams_in, g, sp_in, F, _uncorrected(op))
    assert _rel(plain[2], ref_gF) > 1e-3   # the correction is visible in the force gradient
    sim.close()


@pytest.mark.parametrize("name", ["const", "smag_yu", "implicit_chai"])
def test_loss_seed_with_the_correction(name):
    import torch
    from oracle import adjoint as adj
    from oracle import adjoint_visc as av
    from paper_1704_07559_amd import capi
    shape = (4, 11, 67)
    op, cp, F, g, sp, sim = _adj_setup(name, shape, False, 50)
    N = cp.N
    A = sim.adjoint_planes
    lam = torch.empty((A, N), device="cuda")
    gF = torch.zeros((3, N), device="cuda")
    J = capi.lbm_strain_loss_seed(sim.ctx, lam, gF)
    pf = adj._with_force(op, F)
    if name == "const":
        Jr, lamr, gFr = adj.strain_loss_seed(g, F, pf)
        lamsr = None
        gFp = adj.strain_loss_seed(g, F, _uncorrected(op))[2]
    else:
        Jr, lamr, lamsr, gFr = av.strain_loss_seed_visc(g, sp, F, pf)
        gFp = av.strain_loss_seed_visc(g, sp, F, _uncorrected(op))[3]
    assert abs(J - Jr) < 1e-5 * Jr
    out = to_np(lam).reshape((A,) + shape)
    assert _rel(out[:19], lamr) < 1e-5
    assert _rel(to_np(gF).reshape(gFr.shape), gFr) < 1e-5
    if lamsr is not None:
        assert _rel(out[19], lamsr) < 1e-5
    assert _rel(gFp, gFr) > 1e-3
    sim.close()


@pytest.mark.parametrize("name", ["const", "smag_yu"])
def test_gradient_with_the_correction(name):
    """Checkpointed GPU gradient (20 steps, every 6) of the corrected-strain loss against the
    FP64 oracle on 12 x 13 x 16 nodes."""
    import torch
    from oracle import adjoint as adj
    from paper_1704_07559_amd import autograd as ag
    shape = (12, 13, 16)
    u0 = _f32(synth.spectrum_velocity(shape, seed=1704, u_rms=0.04))
    F = _f32(synth.uniform_random_force(shape, seed=7559, amp=1e-3))
    op, cp, _ = spec_params(shape, tau=0.8, **ADJ_MODELS[name])
    op.force_corrected = True
    cp.strain_force_correction = 1
    nsteps, every = 20, 6
    Jr, gur, gFr = adj.gradient(u0, F, op, nsteps, every=every)
    u0_t = torch.as_tensor(u0.astype(np.float32)).cuda().requires_grad_(True)
    F_t = torch.as_tensor(F.astype(np.float32)).cuda().requires_grad_(True)
    J = ag.strain_loss(u0_t, F_t, ag.StrainLossProblem(cp, nsteps, every))
    J.backward()
    assert abs(J.item() - Jr) < 1e-4 * Jr
    assert _rel(to_np(u0_t.grad), gur) < 1e-4
    assert _rel(to_np(F_t.grad), gFr) < 1e-4
