"""Parity of the HIP D3Q19 path (through the C ABI) with the FP64 oracle.

Tolerances (FP32 arithmetic against FP64): populations 1e-5 relative on the full
distribution f = g + w rho0, strain 1e-4 of the largest strain norm in the field, after
the number of steps each test states. Grids are ragged (not multiples of the 64-wide
wave or of the 256-thread block) so several blocks, partial waves and periodic wraps occur.
"""
import numpy as np
import pytest

import synth
from oracle import closed_forms as cf
from oracle import d3q19 as od
from tests._common import needs_gpu, pop_rel_err, spec_params, strain_rel_err, to_np

pytestmark = [pytest.mark.gpu, needs_gpu]

POP_TOL = 1e-5
STRAIN_TOL = 1e-4


def _lib():
    from paper_1704_07559_amd import capi, lbm
    return capi, lbm


def _smooth_fields(shape, seed, amp=0.03):
    u = synth.random_vector(shape, seed=seed, scale=amp)
    dr = synth.random_vector(shape, seed=seed + 1, scale=0.01)[0]
    grad = synth.random_vector(shape, seed=seed + 2, scale=3e-3).reshape(1, 3, *shape)
    grad = np.concatenate([grad, synth.random_vector(shape, seed=seed + 3, scale=3e-3)[None],
                           synth.random_vector(shape, seed=seed + 4, scale=3e-3)[None]], axis=0)
    return dr, u, grad


@pytest.mark.parametrize("shape", [(5, 11, 37), (3, 70, 129), (1, 1, 1), (2, 3, 300)])
def test_init_then_gather_matches_oracle(shape):
    capi, lbm = _lib()
    dr, u, grad = _smooth_fields(shape, 1)
    op, cp, _ = spec_params(shape, tau=0.7)
    sim = lbm.LBM(cp, lbm.rho_u_field(dr, u), lbm.grad_field(grad))
    g_gpu = to_np(sim.populations())
    g_ref = od.init_populations(dr, u, op, grad)
    assert pop_rel_err(g_gpu, g_ref) < 1e-6


@pytest.mark.parametrize("walls", [False, True])
def test_set_get_roundtrip_is_exact(walls):
    import torch
    capi, lbm = _lib()
    shape = (4, 9, 67)
    op, cp, _ = spec_params(shape, walls=walls)
    sim = lbm.LBM(cp)
    g = torch.as_tensor(synth.random_state(19, shape, seed=3, scale=0.01).astype(np.float32)).cuda()
    sim.set_populations(g)
    assert torch.equal(sim.populations(), g)


CASES = {
    "const": dict(),
    "const_srt": dict(s=np.full(19, 1.0 / 0.9)),
    "const_omegas": dict(omegas=(0.0, -475.0 / 63.0, 0.0)),
    "smag_yu": dict(visc="smagorinsky", drive="yu", nu0=1.0 / 300.0, c_smag=0.1),
    "smag_chai": dict(visc="smagorinsky", drive="chai", nu0=0.01, c_smag=0.3),
    "powerlaw_chai_walls_force": dict(visc="powerlaw", drive="chai", K_pl=0.02, n_pl=0.5, nu_min=1e-3,
                                      nu_max=1.0, walls=True, force=np.array([0.0, 0.0, 1e-5])),
    "powerlaw_yu_shear_thick": dict(visc="powerlaw", drive="yu", K_pl=0.3, n_pl=1.5, nu_min=1e-3, nu_max=1.0),
    "force_field": dict(force="field"),
    "smag_implicit_yu": dict(visc="smagorinsky_implicit", drive="yu", nu0=1.0 / 300.0, c_smag=0.3),
    "smag_implicit_chai_force": dict(visc="smagorinsky_implicit", drive="chai", nu0=0.01, c_smag=0.5, force="field"),
    "rho0_2": dict(rho0=2.0, tau=0.6),
}


# box shapes for the three ways a block pulls along x: whole rows with masked lanes (69),
# whole rows exchanged through LDS (64: 4 rows of 64 per block), part rows (192: 64 wide)
SHAPES = [(4, 10, 69), (3, 8, 64), (2, 5, 192)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("case", sorted(CASES))
def test_steps_from_random_state(case, shape):
    """A far-from-equilibrium random state (every moment non-zero), 3 steps; populations and
    both strain formulas (every step) against the oracle."""
    import torch
    capi, lbm = _lib()
    kw = dict(CASES[case])
    if isinstance(kw.get("force"), str) and kw["force"] == "field":
        kw["force"] = synth.uniform_random_force(shape, seed=7559, amp=1e-4)
    op, cp, _ = spec_params(shape, **kw)
    sim = lbm.LBM(cp)
    g0 = synth.random_state(19, shape, seed=11, scale=3e-3)
    sim.set_populations(torch.as_tensor(g0.astype(np.float32)).cuda())
    ref = od.Simulation(op, g0.astype(np.float32).astype(np.float64))
    S = torch.empty((6,) + shape, device="cuda")
    for n in range(3):
        S_chai = to_np(sim.strain(capi.LBM_STRAIN_CHAI))
        sim.step(1, S_out=S, strain_kind=capi.LBM_STRAIN_YU)
        out = ref.step(1)
        assert strain_rel_err(to_np(S), out.S_yu) < STRAIN_TOL, n
        assert strain_rel_err(S_chai, out.S_chai) < STRAIN_TOL, n
        assert pop_rel_err(to_np(sim.populations()), ref.g, op.rho0) < POP_TOL, n
    if sim.s_nu is not None:
        assert np.max(np.abs(to_np(sim.s_nu).reshape(shape) - ref.s_nu) / ref.s_nu) < 1e-5


@pytest.mark.slow
def test_taylor_green_32_cubed_200_steps():
    """Rotated Taylor-Green vortex, 32^3 periodic, u0 = 0.05, rho0 = 1, tau_nu = 0.8, 200
    steps from the Chapman-Enskog initial state; the Yu strain (emitted by the step) and the
    Chai strain (queried before each step) at every step, the populations at the end, all
    against the FP64 oracle; S_xy also against the closed form."""
    import torch
    capi, lbm = _lib()
    N, tau, u0, steps = 32, 0.8, 0.05, 200
    shape = (N, N, N)
    dr, u, grad = synth.tgv_rotated(shape, u0, 1.0)
    op, cp, _ = spec_params(shape, tau=tau)
    sim = lbm.LBM(cp, lbm.rho_u_field(dr, u), lbm.grad_field(grad))
    ref = od.Simulation(op, od.init_populations(dr, u, op, grad))
    Syu = torch.empty((steps, 6) + shape, device="cuda")
    Sch = torch.empty((steps, 6) + shape, device="cuda")
    for n in range(steps):
        capi.lbm_strain(sim.ctx, capi.LBM_STRAIN_CHAI, Sch[n])
        sim.step(1, S_out=Syu[n], strain_kind=capi.LBM_STRAIN_YU)
    torch.cuda.synchronize()
    worst_yu = worst_chai = 0.0
    for n in range(steps):
        out = ref.step(1)
        worst_yu = max(worst_yu, strain_rel_err(to_np(Syu[n]), out.S_yu))
        worst_chai = max(worst_chai, strain_rel_err(to_np(Sch[n]), out.S_chai))
    assert worst_yu < STRAIN_TOL and worst_chai < STRAIN_TOL, (worst_yu, worst_chai)
    assert pop_rel_err(to_np(sim.populations()), ref.g) < POP_TOL
    for kind, okind in ((capi.LBM_STRAIN_YU, "yu"), (capi.LBM_STRAIN_CHAI, "chai")):
        S = to_np(sim.strain(kind))
        assert strain_rel_err(S, ref.strain(okind)) < STRAIN_TOL
        exact = cf.tgv_rotated_strain(shape, u0, cf.nu_of_rate(1 / tau), steps)
        assert np.linalg.norm(S[3] - exact[3]) / np.linalg.norm(exact[3]) < 5e-3


def test_reduce_matches_oracle_and_flags_nonfinite():
    import torch
    capi, lbm = _lib()
    shape = (6, 13, 41)
    dr, u, grad = _smooth_fields(shape, 5)
    F = synth.uniform_random_force(shape, seed=2, amp=1e-4)
    op, cp, _ = spec_params(shape, visc="smagorinsky", nu0=0.01, force=F)
    sim = lbm.LBM(cp, lbm.rho_u_field(dr, u), lbm.grad_field(grad))
    g0 = od.init_populations(dr, u, op, grad)
    ref = od.Simulation(op, g0)
    sim.step(2)
    ref.step(2)
    d = sim.reduce()
    r = ref.diagnostics()
    assert abs(d["mass"] - r["mass"]) < 1e-6 * np.abs(dr).sum()
    assert np.abs(d["mom"] - r["mom"]).max() < 1e-6 * np.abs(u).sum()
    assert abs(d["ke"] - r["ke"]) < 1e-5 * r["ke"]
    assert abs(d["ss"] - r["ss"]) < 1e-4 * r["ss"]
    assert abs(d["umax"] - r["umax"]) < 1e-5 * r["umax"]
    assert d["nonfinite"] == 0
    # a non-finite population forced from the host is counted and reported
    g = sim.populations()
    g[3, 2, 5, 7] = float("nan")
    sim.set_populations(g)
    with pytest.raises(capi.LBMError) as e:
        sim.reduce()
    assert e.value.status == capi.LBM_ENONFINITE
    assert sim.reduce(allow_nonfinite=True)["nonfinite"] == 1


def test_reduce_is_deterministic_and_conserves():
    capi, lbm = _lib()
    shape = (32, 48, 64)
    dr, u, grad = _smooth_fields(shape, 9, amp=0.02)
    op, cp, _ = spec_params(shape, tau=0.6)
    sim = lbm.LBM(cp, lbm.rho_u_field(dr, u), lbm.grad_field(grad))
    d0 = sim.reduce()
    again = sim.reduce()
    assert all(np.array_equal(np.atleast_1d(again[k]), np.atleast_1d(d0[k])) for k in d0)
    sim.step(100)
    d1 = sim.reduce()
    scale_m = np.abs(dr).sum()
    assert abs(d1["mass"] - d0["mass"]) < 1e-5 * scale_m
    assert np.abs(d1["mom"] - d0["mom"]).max() < 1e-5 * np.abs(u).sum()


def test_error_paths_return_status_without_launching():
    """Unsupported or invalid calls on a live context return a status and leave the state
    untouched (no launch happens)."""
    import torch
    capi, lbm = _lib()
    shape = (4, 6, 64)
    op, cp, _ = spec_params(shape, visc="smagorinsky", nu0=0.01)
    sim = lbm.LBM(cp)
    before = sim.populations().clone()
    N = cp.N
    lam = torch.zeros((sim.adjoint_planes, N), device="cuda")
    rec = torch.zeros((sim.save_planes, N), device="cuda")
    p2 = capi.Params(nx=16, ny=8, nz=1, lattice=capi.LBM_D2Q9, s=[0.0, 1.19, 1.4, 0.0, 1.2, 0.0, 1.2, 1.25, 1.25])
    sim2 = lbm.LBM(p2)
    for call, status in (
        (lambda: capi.lbm_adjoint_step(sim.ctx, None, lam, torch.empty_like(lam)), capi.LBM_EINVAL),
        (lambda: capi.lbm_adjoint_step(sim.ctx, rec, lam, lam), capi.LBM_EINVAL),          # aliasing
        (lambda: capi.lbm_adjoint_step(sim2.ctx, rec, lam, torch.empty_like(lam)), capi.LBM_EUNSUPPORTED),
        (lambda: capi.lbm_strain_loss_seed(sim2.ctx, lam), capi.LBM_EUNSUPPORTED),         # D2Q9
        (lambda: capi.lbm_step(sim2.ctx, 1, None, capi.LBM_STRAIN_YU, rec), capi.LBM_EUNSUPPORTED),
        (lambda: capi.lbm_step(sim.ctx, -1), capi.LBM_EINVAL),
        (lambda: capi.lbm_step(sim.ctx, 1, torch.empty((6, N), device="cuda"), 7), capi.LBM_EINVAL),
        (lambda: capi.lbm_strain(sim.ctx, capi.LBM_STRAIN_YU, None), capi.LBM_EINVAL),
    ):
        with pytest.raises(capi.LBMError) as e:
            call()
        assert e.value.status == status, capi.lbm_last_error()
    sim.step(0)
    assert torch.equal(sim.populations(), before)
    assert sim.step_count == 0
    sim2.close()
    sim.close()


def test_adjoint_lam_aliasing_rejected():
    import torch
    capi, lbm = _lib()
    shape = (4, 6, 64)
    op, cp, _ = spec_params(shape)
    sim = lbm.LBM(cp)
    N = cp.N
    lam = torch.zeros((19, N), device="cuda")
    with pytest.raises(capi.LBMError) as e:
        capi.lbm_adjoint_step(sim.ctx, torch.zeros((3, N), device="cuda"), lam, lam)
    assert e.value.status == capi.LBM_EINVAL


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, 1 << 20, (1 << 22) + 4096 + 48])
def test_stream_copy_is_exact(nbytes):
    """The STREAM-style copy the benchmark uses for context copies every byte, and nothing
    beyond the range (a guard region after the destination keeps its contents)."""
    import torch
    capi, _ = _lib()
    src = torch.randint(-2**31, 2**31 - 1, (nbytes // 4,), dtype=torch.int32, device="cuda")
    dst = torch.full((nbytes // 4 + 64,), 7, dtype=torch.int32, device="cuda")
    capi.lbm_stream_copy(src, dst, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[: nbytes // 4], src)
    assert bool((dst[nbytes // 4:] == 7).all())


@pytest.mark.parametrize("shape,walls", [((1, 1, 1), False), ((1, 2, 1), True), ((2, 1, 3), False),
                                         ((1, 3, 2), True), ((5, 1, 1), False)])
def test_degenerate_boxes(shape, walls):
    """Boxes one or two nodes wide along some axes, where pulled populations wrap onto the node
    itself or its only neighbour (and, with walls, both walls bound the same row): three
    steps with a force field and lagged Smagorinsky against the oracle, and the reduction."""
    import torch
    capi, lbm = _lib()
    F = synth.uniform_random_force(shape, seed=21, amp=1e-4)
    op, cp, _ = spec_params(shape, walls=walls, force=F, visc="smagorinsky", drive="chai", nu0=0.01, c_smag=0.3)
    sim = lbm.LBM(cp)
    g0 = synth.random_state(19, shape, seed=22, scale=3e-3)
    sim.set_populations(torch.as_tensor(g0.astype(np.float32)).cuda())
    ref = od.Simulation(op, g0.astype(np.float32).astype(np.float64))
    S = torch.empty((6,) + shape, device="cuda")
    for n in range(3):
        sim.step(1, S_out=S, strain_kind=capi.LBM_STRAIN_CHAI)
        out = ref.step(1)
        assert strain_rel_err(to_np(S), out.S_chai) < STRAIN_TOL, n
        assert pop_rel_err(to_np(sim.populations()), ref.g, op.rho0) < POP_TOL, n
    d, r = sim.reduce(), ref.diagnostics()
    assert abs(d["mass"] - r["mass"]) < 1e-6 and np.abs(np.asarray(d["mom"]) - r["mom"]).max() < 1e-6
    assert abs(d["ss"] - r["ss"]) < 1e-4 * r["ss"]
    sim.close()


def test_reduce_async_matches_reduce():
    """The non-blocking diagnostics give the blocking call's bits, into pinned host memory
    and into device memory, also when queued between steps and read afterwards."""
    import torch
    capi, lbm = _lib()
    shape = (6, 10, 64)
    dr, u, grad = _smooth_fields(shape, 31)
    op, cp, _ = spec_params(shape, visc="smagorinsky", nu0=0.01, c_smag=0.2)
    sim = lbm.LBM(cp, lbm.rho_u_field(dr, u), lbm.grad_field(grad))
    host = torch.zeros((3, 8), dtype=torch.float64, pin_memory=True)
    dev = torch.zeros((3, 8), dtype=torch.float64, device="cuda")
    ref = []
    for k in range(3):
        sim.step(2)
        sim.reduce_async(host[k])
        sim.reduce_async(dev[k])
        torch.cuda.current_stream().synchronize()
        ref.append(capi.lbm_reduce(sim.ctx))
    for k in range(3):
        assert host[k].tolist() == ref[k]
        assert dev[k].cpu().tolist() == ref[k]
    # queued between steps, read only at the end
    a = lbm.LBM(cp, lbm.rho_u_field(dr, u), lbm.grad_field(grad))
    slots = torch.zeros((3, 8), dtype=torch.float64, pin_memory=True)
    for k in range(3):
        a.step(2)
        a.reduce_async(slots[k])
    torch.cuda.current_stream().synchronize()
    assert [slots[k].tolist() for k in range(3)] == ref
    sim.close()
    a.close()


@pytest.mark.parametrize("c_smag,scale", [(1.0, 0.05), (2.0, 0.2), (0.05, 0.2)])
def test_implicit_smagorinsky_extreme_strain(c_smag, scale):
    """The implicit coupling's fixed Newton solve far from the LES regime: large C_s and
    strongly non-equilibrium states (strain magnitudes up to O(1)), where the initial guess
    (the root without the isotropic part) is farthest from the solution. One step against
    the oracle's bisection."""
    import torch
    capi, lbm = _lib()
    shape = (3, 8, 64)
    op, cp, _ = spec_params(shape, tau=0.9, visc="smagorinsky_implicit", drive="yu", nu0=1e-4, c_smag=c_smag)
    g0 = synth.random_state(19, shape, seed=23, scale=scale).astype(np.float32).astype(np.float64)
    sim = lbm.LBM(cp)
    sim.set_populations(torch.as_tensor(g0.astype(np.float32)).cuda())
    ref = od.Simulation(op, g0)
    S = torch.empty((6,) + shape, device="cuda")
    sim.step(1, S_out=S, strain_kind=capi.LBM_STRAIN_YU)
    out = ref.step(1)
    assert strain_rel_err(to_np(S), out.S_yu) < STRAIN_TOL
    # these states have populations near zero and below it, so the error is normalised by the
    # largest deviation rather than elementwise by f
    g = to_np(sim.populations())
    assert np.abs(g - ref.g).max() / np.abs(ref.g).max() < POP_TOL
    sim.close()
