"""Parity of the hand-written adjoint kernels (through the C ABI) with the FP64 adjoint
oracle, and of the checkpointed torch.autograd.Function with the oracle gradient.

Tolerances: adjoint quantities are compared field-normalised, max|d| / max|ref| <= 1e-5
for one kernel call (FP32 against FP64) and <= 1e-4 for whole gradients over tens of
steps; the directional derivatives (accumulated in FP64) to 1e-4 relative.
"""
import numpy as np
import pytest

import synth
from oracle import adjoint as adj
from oracle import d3q19 as od
from tests._common import needs_gpu, spec_params, to_np

pytestmark = [pytest.mark.gpu, needs_gpu]


def _rel(a, b):
    return float(np.abs(np.asarray(a, dtype=np.float64) - b).max() / np.abs(b).max())


def _state(shape, seed, p):
    u = synth.random_vector(shape, seed=seed, scale=0.03)
    g = od.init_populations(np.zeros(shape), u, p) + synth.random_state(19, shape, seed=seed + 1, scale=2e-3)
    return g.astype(np.float32).astype(np.float64)


# (5, 9, 70): blocks of whole rows with masked lanes; (3, 8, 64): whole rows of 64, the
# x-shifted adjoint elements exchanged through LDS
@pytest.mark.parametrize("shape", [(5, 9, 70), (3, 8, 64)])
@pytest.mark.parametrize("walls", [False, True])
def test_adjoint_step_matches_oracle(walls, shape):
    import torch
    from paper_1704_07559_amd import capi, lbm
    F = synth.uniform_random_force(shape, seed=3, amp=1e-4)
    op, cp, _ = spec_params(shape, tau=0.7, walls=walls, force=F)
    g = _state(shape, 1, op)
    sim = lbm.LBM(cp)
    sim.set_populations(torch.as_tensor(g.astype(np.float32)).cuda())
    N = cp.N
    jbuf = torch.empty((1, 3, N), device="cuda")
    sim.step(1, save=jbuf)      # saves j of the collision of state g
    lam_in = synth.random_state(19, shape, seed=4, scale=1.0)
    lam_t = torch.as_tensor(lam_in.astype(np.float32)).cuda().reshape(19, N).contiguous()
    lam_out = torch.empty_like(lam_t)
    gF = torch.zeros((3, N), device="cuda")
    capi.lbm_adjoint_step(sim.ctx, jbuf[0], lam_t, lam_out, gF)
    ref_lam, ref_gF = adj.adjoint_step(lam_in.astype(np.float32).astype(np.float64), g, F, op)
    assert _rel(to_np(lam_out).reshape(ref_lam.shape), ref_lam) < 1e-5
    assert _rel(to_np(gF).reshape(ref_gF.shape), ref_gF) < 1e-5


def test_loss_seed_and_init_adjoint_match_oracle():
    import torch
    from paper_1704_07559_amd import capi, lbm
    shape = (4, 11, 67)
    F = synth.uniform_random_force(shape, seed=5, amp=1e-4)
    op, cp, _ = spec_params(shape, tau=0.75, force=F)
    g = _state(shape, 6, op)
    sim = lbm.LBM(cp)
    sim.set_populations(torch.as_tensor(g.astype(np.float32)).cuda())
    N = cp.N
    lam = torch.empty((19, N), device="cuda")
    gF = torch.zeros((3, N), device="cuda")
    J = capi.lbm_strain_loss_seed(sim.ctx, lam, gF)
    Jr, lamr, gFr = adj.strain_loss_seed(g, F, op)
    assert abs(J - Jr) < 1e-5 * Jr
    assert _rel(to_np(lam).reshape(lamr.shape), lamr) < 1e-5
    assert _rel(to_np(gF).reshape(gFr.shape), gFr) < 1e-5
    u0 = synth.random_vector(shape, seed=7, scale=0.04)
    rho_u = torch.as_tensor(np.concatenate([np.zeros((1,) + shape), u0]).astype(np.float32)).cuda().reshape(4, N)
    lam0 = synth.random_state(19, shape, seed=8, scale=1.0)
    gu = torch.empty((3, N), device="cuda")
    capi.lbm_init_adjoint(sim.ctx, rho_u, torch.as_tensor(lam0.astype(np.float32)).cuda().reshape(19, N), gu)
    ref = adj.init_adjoint(lam0.astype(np.float32).astype(np.float64), u0.astype(np.float32).astype(np.float64), op)
    assert _rel(to_np(gu).reshape(ref.shape), ref) < 1e-5


def _c4(n):
    shape = (n, n, n)
    u0 = synth.spectrum_velocity(shape, seed=1704, u_rms=0.04)
    F = synth.uniform_random_force(shape, seed=7559, amp=1e-6)
    return shape, u0, F


@pytest.mark.parametrize("nsteps,every", [(50, 10), (23, 7)])
def test_strain_loss_gradient_16_cubed(nsteps, every):
    """The C4 recipe on 16^3: checkpointed GPU gradient against the FP64 oracle gradient."""
    import torch
    from paper_1704_07559_amd import autograd as ag
    shape, u0, F = _c4(16)
    op, cp, _ = spec_params(shape, tau=0.8)
    Jr, gur, gFr = adj.gradient(u0, F, op, nsteps, every=every)
    u0_t = torch.as_tensor(u0.astype(np.float32)).cuda().requires_grad_(True)
    F_t = torch.as_tensor(F.astype(np.float32)).cuda().requires_grad_(True)
    J = ag.strain_loss(u0_t, F_t, ag.StrainLossProblem(cp, nsteps, every))
    J.backward()
    assert abs(J.item() - Jr) < 1e-4 * Jr
    gu, gF = to_np(u0_t.grad), to_np(F_t.grad)
    assert _rel(gu, gur) < 1e-4
    assert _rel(gF, gFr) < 1e-4
    d = synth.random_vector(shape, seed=3, scale=1.0)
    dd = torch.as_tensor(d).cuda()
    assert abs((u0_t.grad.double() * dd).sum().item() - (gur * d).sum()) < 1e-4 * abs((gur * d).sum())
    assert abs((F_t.grad.double() * dd).sum().item() - (gFr * d).sum()) < 1e-4 * abs((gFr * d).sum())


@pytest.mark.parametrize("visc,nsteps", [("const", 21), ("smagorinsky", 21), ("const", 0)])
def test_checkpoint_interval_does_not_change_the_gradient(visc, nsteps):
    """Recompute is bit-identical on the GPU too: the gradient with checkpoints every 7 steps
    equals the gradient with one checkpoint, and both equal the gradient from records kept
    by the forward sweep (no recompute), for a constant and a lagged viscosity, and for a
    run of no steps (the loss of the initial state)."""
    import torch
    from paper_1704_07559_amd import autograd as ag
    shape, u0, F = _c4(12)
    kw = {} if visc == "const" else dict(visc="smagorinsky", drive="yu", nu0=0.01, c_smag=0.3)
    op, cp, _ = spec_params(shape, tau=0.8, **kw)
    grads = []
    for every, record_all in ((21, False), (7, False), (50, True)):
        u0_t = torch.as_tensor(u0.astype(np.float32)).cuda().requires_grad_(True)
        F_t = torch.as_tensor(F.astype(np.float32)).cuda().requires_grad_(True)
        J = ag.strain_loss(u0_t, F_t, ag.StrainLossProblem(cp, nsteps, every, record_all=record_all))
        J.backward()
        grads.append((J.item(), u0_t.grad.clone(), F_t.grad.clone()))
    for g in grads[1:]:
        assert g[0] == grads[0][0] and torch.equal(g[1], grads[0][1]) and torch.equal(g[2], grads[0][2])


def test_strain_loss_gradient_500_steps_against_stored_oracle():
    """The adjoint recipe at its full length on 16^3: 500 steps, checkpoint every 50, against
    the FP64 oracle gradient stored by tests/golden/make_adjoint_golden.py."""
    import pathlib

    import torch
    from paper_1704_07559_amd import autograd as ag
    ref = np.load(pathlib.Path(__file__).parent / "golden" / "adjoint_c4_16cubed_500.npz")
    shape, u0, F = _c4(16)
    op, cp, _ = spec_params(shape, tau=0.8)
    u0_t = torch.as_tensor(u0.astype(np.float32)).cuda().requires_grad_(True)
    F_t = torch.as_tensor(F.astype(np.float32)).cuda().requires_grad_(True)
    J = ag.strain_loss(u0_t, F_t, ag.StrainLossProblem(cp, int(ref["steps"]), int(ref["every"])))
    J.backward()
    assert abs(J.item() - float(ref["J"])) < 1e-4 * float(ref["J"])
    assert _rel(to_np(u0_t.grad), ref["grad_u0"]) < 1e-4
    assert _rel(to_np(F_t.grad), ref["grad_F"]) < 1e-4


def test_gpu_gradient_against_gpu_finite_differences():
    """Directional derivatives of the GPU loss (FP32 states, J accumulated in FP64) by the
    five-point central difference, against the GPU adjoint gradient (16^3, 40 steps)."""
    import torch
    from paper_1704_07559_amd import autograd as ag
    shape, u0, F = _c4(16)
    op, cp, _ = spec_params(shape, tau=0.8)
    prob = ag.StrainLossProblem(cp, 40, 10)
    u0_t = torch.as_tensor(u0.astype(np.float32)).cuda().requires_grad_(True)
    F_t = torch.as_tensor(F.astype(np.float32)).cuda().requires_grad_(True)
    ag.strain_loss(u0_t, F_t, prob).backward()
    du = torch.as_tensor(synth.random_vector(shape, seed=5, scale=1.0).astype(np.float32)).cuda()
    dF = torch.as_tensor(synth.random_vector(shape, seed=6, scale=1.0).astype(np.float32)).cuda()

    def J(u, f):
        with torch.no_grad():
            return ag.strain_loss(u, f, prob).item()

    def fd5(fun, h):
        return (8 * (fun(h) - fun(-h)) - (fun(2 * h) - fun(-2 * h))) / (12 * h)

    u_d, F_d = u0_t.detach(), F_t.detach()
    hu = 1e-3 * float(u_d.abs().max())
    hF = 1e-5  # |F| ~ 1e-6: a larger step keeps the FP32 rounding of J far below the signal
    fd_u = fd5(lambda t: J(u_d + t * du, F_d), hu)
    fd_F = fd5(lambda t: J(u_d, F_d + t * dF), hF)
    ad_u = float((u0_t.grad.double() * du.double()).sum())
    ad_F = float((F_t.grad.double() * dF.double()).sum())
    assert abs(fd_u - ad_u) < 1e-3 * abs(ad_u), (fd_u, ad_u)
    assert abs(fd_F - ad_F) < 1e-3 * abs(ad_F), (fd_F, ad_F)


@pytest.mark.slow
def test_adjoint_step_128_cubed_sampled_against_oracle():
    """The adjoint kernel at the benchmarked size (128^3, force field, constant viscosity),
    in that launch configuration: one reverse step from a random far-from-equilibrium
    state and a random adjoint state, checked at sampled nodes against the FP64 oracle
    evaluated on each node's 3 x 3 x 3 neighbourhood (the step at a node reads no other
    node)."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    from tests._common import sample_nodes
    n = 128
    shape = (n, n, n)
    F = synth.uniform_random_force(shape, seed=7559, amp=1e-6).astype(np.float32).astype(np.float64)
    op, cp, _ = spec_params(shape, tau=0.8, force=F)
    g = _state(shape, 21, op)
    sim = lbm.LBM(cp)
    sim.set_populations(torch.as_tensor(g.astype(np.float32)).cuda())
    N = cp.N
    rec = torch.empty((1, 3, N), device="cuda")
    sim.step(1, save=rec)
    lam = synth.random_state(19, shape, seed=22, scale=1.0).astype(np.float32).astype(np.float64)
    lam_t = torch.as_tensor(lam.astype(np.float32)).cuda().reshape(19, N)
    out = torch.empty_like(lam_t)
    gF = torch.zeros((3, N), device="cuda")
    capi.lbm_adjoint_step(sim.ctx, rec[0], lam_t, out, gF)
    out = out.reshape((19,) + shape)
    gF = gF.reshape((3,) + shape)
    worst, worst_F = 0.0, 0.0
    scale, scale_F = 0.0, 0.0
    for (z, y, x) in sample_nodes(shape, 30, 23):
        ix = np.ix_([(z + d) % n for d in (-1, 0, 1)], [(y + d) % n for d in (-1, 0, 1)],
                    [(x + d) % n for d in (-1, 0, 1)])
        gp = np.stack([g[i][ix] for i in range(19)])
        lp = np.stack([lam[i][ix] for i in range(19)])
        Fp = np.stack([F[c][ix] for c in range(3)])
        ref_l, ref_F = adj.adjoint_step(lp, gp, Fp, adj._with_force(op, Fp))
        got = out[:, z, y, x].double().cpu().numpy()
        got_F = gF[:, z, y, x].double().cpu().numpy()
        worst = max(worst, float(np.abs(got - ref_l[:, 1, 1, 1]).max()))
        worst_F = max(worst_F, float(np.abs(got_F - ref_F[:, 1, 1, 1]).max()))
        scale = max(scale, float(np.abs(ref_l[:, 1, 1, 1]).max()))
        scale_F = max(scale_F, float(np.abs(ref_F[:, 1, 1, 1]).max()))
    assert worst < 1e-5 * scale and worst_F < 1e-5 * scale_F, (worst / scale, worst_F / scale_F)
    sim.close()


@pytest.mark.slow
def test_gradient_128_cubed_500_steps_against_gpu_finite_differences():
    """The whole benchmarked gradient (128^3, 500 steps, checkpoint every 50): directional
    derivatives of J by five-point central differences of the GPU forward, a property that
    holds at any size, against the adjoint gradient."""
    import torch
    from paper_1704_07559_amd import autograd as ag
    shape, u0, F = _c4(128)
    op, cp, _ = spec_params(shape, tau=0.8)
    prob = ag.StrainLossProblem(cp, 500, 50)
    u0_t = torch.as_tensor(u0.astype(np.float32)).cuda().requires_grad_(True)
    F_t = torch.as_tensor(F.astype(np.float32)).cuda().requires_grad_(True)
    ag.strain_loss(u0_t, F_t, prob).backward()
    du = torch.as_tensor(synth.random_vector(shape, seed=5, scale=1.0).astype(np.float32)).cuda()
    dF = torch.as_tensor(synth.random_vector(shape, seed=6, scale=1.0).astype(np.float32)).cuda()

    def J(u, f):
        with torch.no_grad():
            return ag.strain_loss(u, f, prob).item()

    def fd5(fun, h):
        return (8 * (fun(h) - fun(-h)) - (fun(2 * h) - fun(-2 * h))) / (12 * h)

    u_d, F_d = u0_t.detach(), F_t.detach()
    fd_u = fd5(lambda t: J(u_d + t * du, F_d), 1e-3 * float(u_d.abs().max()))
    fd_F = fd5(lambda t: J(u_d, F_d + t * dF), 1e-5)
    ad_u = float((u0_t.grad.double() * du.double()).sum())
    ad_F = float((F_t.grad.double() * dF.double()).sum())
    assert abs(fd_u - ad_u) < 2e-3 * abs(ad_u), (fd_u, ad_u)
    assert abs(fd_F - ad_F) < 2e-3 * abs(ad_F), (fd_F, ad_F)


@pytest.mark.parametrize("storage,tol", [("f16", 2e-2), ("bf16", 1e-1)])
def test_strain_loss_gradient_with_half_storage(storage, tol):
    """The checkpointed gradient with FP16 / BF16 population storage (all arithmetic FP32,
    the adjoint the transpose of that arithmetic at the stored states) against the FP64
    oracle gradient of the unrounded forward, C4 recipe on 16^3, 50 steps: a stated error
    of the order of the storage rounding accumulated over the run (no reference exists for
    the rounded trajectory itself). The recompute is also exact in reduced storage: two
    checkpoint intervals give the same bits."""
    import torch
    from paper_1704_07559_amd import autograd as ag
    shape, u0, F = _c4(16)
    op, cp, _ = spec_params(shape, tau=0.8, storage=storage)
    nsteps = 50
    Jr, gur, gFr = adj.gradient(u0, F, op, nsteps, every=10)
    grads = []
    for every in (10, 7):
        u0_t = torch.as_tensor(u0.astype(np.float32)).cuda().requires_grad_(True)
        F_t = torch.as_tensor(F.astype(np.float32)).cuda().requires_grad_(True)
        J = ag.strain_loss(u0_t, F_t, ag.StrainLossProblem(cp, nsteps, every))
        J.backward()
        grads.append((J.item(), to_np(u0_t.grad), to_np(F_t.grad)))
    J, gu, gF = grads[0]
    assert abs(J - Jr) < tol * Jr
    assert _rel(gu, gur) < tol and _rel(gF, gFr) < tol, (_rel(gu, gur), _rel(gF, gFr))
    assert grads[1][0] == J and np.array_equal(grads[1][1], gu) and np.array_equal(grads[1][2], gF)
