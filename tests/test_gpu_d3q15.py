"""Parity of the HIP D3Q15 path (through the C ABI) with the FP64 D3Q15 oracle.

Same tolerances as the D3Q19 tests: populations 1e-5 relative on f = g + w rho0, strain
1e-4 of the largest strain norm in the field."""
import numpy as np
import pytest

import synth
from oracle import closed_forms as cf
from oracle import d3q15 as od
from tests._common import needs_gpu, pop_rel_err, strain_rel_err, to_np

pytestmark = [pytest.mark.gpu, needs_gpu]


def _spec(shape, tau=0.8, s=None, visc="const", drive="yu", walls=False, force=None, storage=0, **kw):
    import torch
    from paper_1704_07559_amd import capi
    nz, ny, nx = shape
    sv = od.default_rates(tau) if s is None else np.asarray(s, dtype=np.float64)
    op = od.Params(s=sv.copy(), visc_kind=visc, visc_strain=drive, walls_y=walls, force=force, **kw)
    vk = {"const": 0, "smagorinsky": 1, "powerlaw": 2, "smagorinsky_implicit": 3}[visc]
    fvec, ft = (0.0, 0.0, 0.0), None
    if force is not None:
        F = np.asarray(force, dtype=np.float64)
        if F.shape == (3,):
            fvec = tuple(float(v) for v in F)
        else:
            ft = torch.as_tensor(F.reshape(3, -1).astype(np.float32)).cuda().contiguous()
    cp = capi.Params(nx=nx, ny=ny, nz=nz, lattice=capi.LBM_D3Q15, storage=storage, walls_y=int(walls),
                     s=list(sv) + [0.0] * 4, visc_kind=vk, visc_strain=1 if drive == "yu" else 2, force=fvec,
                     force_field=ft, **kw)
    return op, cp


def _pop_err(g_gpu, g_ref):
    return pop_rel_err(g_gpu, g_ref, 1.0, od.W)


@pytest.mark.parametrize("shape", [(5, 11, 37), (3, 70, 129), (1, 1, 1)])
def test_init_then_gather_matches_oracle(shape):
    from paper_1704_07559_amd import lbm
    u = synth.random_vector(shape, seed=1, scale=0.03)
    dr = synth.random_vector(shape, seed=2, scale=0.01)[0]
    grad = np.stack([synth.random_vector(shape, seed=3 + a, scale=3e-3) for a in range(3)])
    op, cp = _spec(shape, tau=0.7)
    sim = lbm.LBM(cp, lbm.rho_u_field(dr, u), lbm.grad_field(grad))
    assert _pop_err(to_np(sim.populations()), od.init_populations(dr, u, op, grad)) < 1e-6
    sim.close()


CASES = {
    "const": dict(),
    "srt": dict(s=np.full(15, 1 / 0.9)),
    "smag_yu": dict(visc="smagorinsky", drive="yu", nu0=0.01, c_smag=0.2),
    "smag_chai_walls": dict(visc="smagorinsky", drive="chai", nu0=0.005, c_smag=0.3, walls=True),
    "powerlaw_chai_walls_force": dict(visc="powerlaw", drive="chai", K_pl=0.02, n_pl=0.6, walls=True,
                                      force=np.array([0.0, 0.0, 1e-5])),
    "force_field": dict(force="field"),
    "smag_implicit_yu": dict(visc="smagorinsky_implicit", drive="yu", nu0=0.002, c_smag=0.3),
    "smag_implicit_chai_walls_force": dict(visc="smagorinsky_implicit", drive="chai", nu0=0.005, c_smag=0.2,
                                           walls=True, force=np.array([1e-5, 0.0, 0.0])),
}


@pytest.mark.parametrize("shape", [(7, 23, 131), (3, 8, 64), (2, 5, 192)])
@pytest.mark.parametrize("case", sorted(CASES))
def test_steps_from_random_state(case, shape):
    """Three steps from a far-from-equilibrium state: the Yu-type strain emitted by the step,
    the Chai strain queried before it, populations and s_nu. The shapes take the three ways a
    block pulls along x (whole rows with masked lanes, whole rows through LDS, part rows)."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    kw = dict(CASES[case])
    if isinstance(kw.get("force"), str):
        kw["force"] = synth.uniform_random_force(shape, seed=5, amp=1e-4)
    op, cp = _spec(shape, **kw)
    sim = lbm.LBM(cp)
    g0 = synth.random_state(15, shape, seed=11, scale=3e-3).astype(np.float32).astype(np.float64)
    sim.set_populations(torch.as_tensor(g0.astype(np.float32)).cuda())
    ref = od.Simulation(op, g0)
    S = torch.empty((6,) + shape, device="cuda")
    for n in range(3):
        S_chai = to_np(sim.strain(capi.LBM_STRAIN_CHAI))
        sim.step(1, S_out=S, strain_kind=capi.LBM_STRAIN_YU)
        Sy, Sc = ref.step(1)
        assert strain_rel_err(to_np(S), Sy) < 1e-4, n
        assert strain_rel_err(S_chai, Sc) < 1e-4, n
        assert _pop_err(to_np(sim.populations()), ref.g) < 1e-5, n
    if sim.s_nu is not None:
        assert np.max(np.abs(to_np(sim.s_nu).reshape(shape) - ref.s_nu) / ref.s_nu) < 1e-5
    d, r = sim.reduce(), ref.diagnostics()
    assert abs(d["ss"] - r["ss"]) < 1e-4 * r["ss"]
    sim.close()


def test_taylor_green_32_cubed_200_steps():
    """Rotated Taylor-Green vortex on D3Q15, 32^3, u0 = 0.05, tau_nu = 0.8, 200 steps from the
    Chapman-Enskog state: strain every 50 steps against the oracle, S_xy against the closed
    form, diagnostics against the oracle."""
    from paper_1704_07559_amd import capi, lbm
    N, tau, u0, steps = 32, 0.8, 0.05, 200
    shape = (N, N, N)
    dr, u, gu = synth.tgv_rotated(shape, u0, 1.0)
    op, cp = _spec(shape, tau=tau)
    sim = lbm.LBM(cp, lbm.rho_u_field(dr, u), lbm.grad_field(gu))
    ref = od.Simulation(op, od.init_populations(dr, u, op, gu))
    for _ in range(4):
        sim.step(50)
        ref.step(50)
        for kind, okind in ((capi.LBM_STRAIN_YU, "yu"), (capi.LBM_STRAIN_CHAI, "chai")):
            assert strain_rel_err(to_np(sim.strain(kind)), ref.strain(okind)) < 1e-4
    assert _pop_err(to_np(sim.populations()), ref.g) < 1e-5
    exact = cf.tgv_rotated_strain(shape, u0, cf.nu_of_rate(1 / tau), steps)[3]
    S = to_np(sim.strain(capi.LBM_STRAIN_YU))[3]
    assert np.linalg.norm(S - exact) / np.linalg.norm(exact) < 5e-3
    d, r = sim.reduce(), ref.diagnostics()
    assert d["nonfinite"] == 0
    assert abs(d["mass"] - r["mass"]) < 1e-5 * np.abs(dr).sum()
    assert abs(d["ke"] - r["ke"]) < 1e-5 * r["ke"]
    assert abs(d["ss"] - r["ss"]) < 1e-4 * r["ss"]
    sim.close()


@pytest.mark.parametrize("storage,tol", [(1, 3e-3), (2, 2e-2)])
def test_half_precision_storage_against_oracle(storage, tol):
    """FP16 / BF16 storage of the deviation g on a 16^3 LES-like field, 20 steps, strain
    against the FP64 oracle within the rounding of the stored deviation."""
    from paper_1704_07559_amd import capi, lbm
    shape = (16, 16, 16)
    u = synth.spectrum_velocity(shape, seed=1704, u_rms=0.04)
    op, cp = _spec(shape, tau=0.6, storage=storage, visc="smagorinsky", nu0=(0.6 - 0.5) / 3, c_smag=0.1)
    sim = lbm.LBM(cp, lbm.rho_u_field(np.zeros(shape), u))
    ref = od.Simulation(op, od.init_populations(np.zeros(shape), u, op))
    sim.step(20)
    ref.step(20)
    assert strain_rel_err(to_np(sim.strain(capi.LBM_STRAIN_YU)), ref.strain("yu")) < tol
    sim.close()


@pytest.mark.slow
def test_les_256_cubed_d3q15_sampled():
    """The D3Q15 LES workload bench.py times (256^3, FP32, Smagorinsky C_s = 0.1 from the
    Yu-type strain, tau_nu0 = 0.51), in that launch configuration: 16 steps, then the
    populations and both strains at sampled nodes against the FP64 oracle run on each node's
    neighbourhood, Yu-type = Chai over the whole field, mass conservation."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    from tests._common import patch_reference, sample_nodes
    n, K = 256, 16
    shape = (n, n, n)
    u = synth.spectrum_velocity(shape, seed=1704, u_rms=0.04)
    kw = dict(visc="smagorinsky", drive="yu", nu0=(0.51 - 0.5) / 3.0, c_smag=0.1)
    op, cp = _spec(shape, tau=0.51, **kw)
    sim = lbm.LBM(cp, lbm.rho_u_field(np.zeros(shape), u))
    m0 = sim.reduce()["mass"]
    S = [torch.empty((6,) + shape, device="cuda") for _ in range(K)]
    for k in range(K):
        sim.step(1, S_out=S[k], strain_kind=capi.LBM_STRAIN_YU)
    Sy, Sc = sim.strain(capi.LBM_STRAIN_YU), sim.strain(capi.LBM_STRAIN_CHAI)
    frob = torch.sqrt((Sy[:3] ** 2).sum(0) + 2 * (Sy[3:] ** 2).sum(0)).max().item()
    assert (Sy - Sc).abs().max().item() < 1e-4 * frob   # two FP32 evaluations of one quantity
    g = sim.populations()
    nodes = sample_nodes(shape, 24, 7)
    idx = tuple(torch.tensor(a, device="cuda") for a in zip(*nodes))
    g_s = g[(slice(None),) + idx].double().cpu().numpy()
    S_s = [s[(slice(None),) + idx].double().cpu().numpy() for s in S]
    d = sim.reduce()
    sim.close()

    def make_params(Fp):
        q = od.Params(**{f: getattr(op, f) for f in op.__dataclass_fields__})
        q.force = Fp
        return q

    worst_g, dS, fr = 0.0, 0.0, 0.0
    wts = np.array([1, 1, 1, 2, 2, 2])
    for m, node in enumerate(nodes):
        g_ref, S_ref, _ = patch_reference(make_params, u, node, K, False, None, oracle=od)
        f_ref = g_ref + od.W
        worst_g = max(worst_g, float(np.max(np.abs(g_s[:, m] + od.W - f_ref) / np.abs(f_ref))))
        for k in range(K):
            dS = max(dS, float(np.abs(S_s[k][:, m] - S_ref[k]).max()))
            fr = max(fr, float(np.sqrt((wts * S_ref[k] ** 2).sum())))
    assert worst_g < 1e-5 and dS / fr < 1e-4, (worst_g, dS / fr)
    assert d["nonfinite"] == 0 and abs(d["mass"] - m0) < 1e-3


@pytest.mark.parametrize("shape,walls", [((1, 1, 1), False), ((1, 2, 1), True), ((2, 1, 3), False), ((3, 2, 1), True)])
def test_degenerate_boxes(shape, walls):
    """Boxes one or two nodes wide along some axes (populations wrap onto the node itself or
    its only neighbour): three steps with a force field and lagged Smagorinsky against the
    oracle."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    F = synth.uniform_random_force(shape, seed=21, amp=1e-4)[:3]
    op, cp = _spec(shape, walls=walls, force=F, visc="smagorinsky", drive="chai", nu0=0.01, c_smag=0.3)
    sim = lbm.LBM(cp)
    g0 = synth.random_state(15, shape, seed=22, scale=3e-3).astype(np.float32).astype(np.float64)
    sim.set_populations(torch.as_tensor(g0.astype(np.float32)).cuda())
    ref = od.Simulation(op, g0)
    S = torch.empty((6,) + shape, device="cuda")
    for n in range(3):
        sim.step(1, S_out=S, strain_kind=capi.LBM_STRAIN_CHAI)
        Sy, Sc = ref.step(1)
        assert strain_rel_err(to_np(S), Sc) < 1e-4, n
        assert _pop_err(to_np(sim.populations()), ref.g) < 1e-5, n
    sim.close()
