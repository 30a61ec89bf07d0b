"""Parity of the HIP D2Q9 path (through the C ABI) with the FP64 D2Q9 oracle.

Same tolerances as the D3Q19 tests: populations 1e-5 relative on f = g + w rho0, strain
1e-4 of the largest strain norm in the field."""
import numpy as np
import pytest

import synth
from oracle import closed_forms as cf
from oracle import d2q9 as od
from tests._common import needs_gpu, pop_rel_err, strain_rel_err, to_np

pytestmark = [pytest.mark.gpu, needs_gpu]


def _spec(shape, tau=0.8, s=None, visc="const", drive="yu", walls=False, force=None, **kw):
    import torch
    from paper_1704_07559_amd import capi
    _, ny, nx = shape
    sv = od.default_rates(tau) if s is None else np.asarray(s, dtype=np.float64)
    op = od.Params(s=sv.copy(), visc_kind=visc, visc_strain=drive, walls_y=walls, force=force, **kw)
    vk = {"const": 0, "smagorinsky": 1, "powerlaw": 2, "smagorinsky_implicit": 3}[visc]
    fvec, ft = (0.0, 0.0, 0.0), None
    if force is not None:
        F = np.asarray(force, dtype=np.float64)
        if F.shape == (2,):
            fvec = (float(F[0]), float(F[1]), 0.0)
        else:
            F3 = np.concatenate([F.reshape(2, -1), np.zeros((1, nx * ny))])
            ft = torch.as_tensor(F3.astype(np.float32)).cuda().contiguous()
    cp = capi.Params(nx=nx, ny=ny, nz=1, lattice=capi.LBM_D2Q9, walls_y=int(walls), s=list(sv) + [0.0] * 10,
                     visc_kind=vk, visc_strain=1 if drive == "yu" else 2, force=fvec, force_field=ft,
                     **{k: v for k, v in kw.items()})
    return op, cp


def _pop_err(g_gpu, g_ref):
    return pop_rel_err(g_gpu, g_ref, 1.0, od.W)


def test_init_then_gather_matches_oracle():
    from paper_1704_07559_amd import lbm
    shape = (1, 37, 300)
    u = synth.random_vector(shape, seed=1, scale=0.03)[:2]
    dr = synth.random_vector(shape, seed=2, scale=0.01)[0]
    grad = np.stack([synth.random_vector(shape, seed=3, scale=3e-3), synth.random_vector(shape, seed=4, scale=3e-3),
                     np.zeros((3,) + shape)])  # grad[a, b] = d u_b / d x_a; the z row and column unused
    op, cp = _spec(shape, tau=0.7)
    sim = lbm.LBM(cp, lbm.rho_u_field(dr, u), lbm.grad_field(grad))
    assert _pop_err(to_np(sim.populations()), od.init_populations(dr, u, op, grad[:2, :2])) < 1e-6


CASES = {
    "const": dict(),
    "srt": dict(s=np.full(9, 1 / 0.9)),
    "smag_yu": dict(visc="smagorinsky", drive="yu", nu0=0.01, c_smag=0.2),
    "powerlaw_chai_walls_force": dict(visc="powerlaw", drive="chai", K_pl=0.02, n_pl=0.6, walls=True,
                                      force=np.array([1e-5, 0.0])),
    "force_field": dict(force="field"),
    "smag_implicit_yu": dict(visc="smagorinsky_implicit", drive="yu", nu0=0.002, c_smag=0.3),
    "smag_implicit_chai_walls_force": dict(visc="smagorinsky_implicit", drive="chai", nu0=0.005, c_smag=0.2,
                                           walls=True, force=np.array([1e-5, 0.0])),
}


@pytest.mark.parametrize("shape", [(1, 23, 131), (1, 8, 128), (1, 5, 320)])
@pytest.mark.parametrize("case", sorted(CASES))
def test_steps_from_random_state(case, shape):
    """Three steps from a far-from-equilibrium state; the shapes take the three ways a block
    pulls along x (whole rows with masked lanes, whole rows through LDS, part rows)."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    kw = dict(CASES[case])
    if isinstance(kw.get("force"), str):
        kw["force"] = synth.uniform_random_force(shape, seed=5, amp=1e-4)[:2]
    op, cp = _spec(shape, **kw)
    sim = lbm.LBM(cp)
    g0 = synth.random_state(9, shape, seed=11, scale=3e-3).astype(np.float32).astype(np.float64)
    sim.set_populations(torch.as_tensor(g0.astype(np.float32)).cuda())
    ref = od.Simulation(op, g0)
    S = torch.empty((3,) + shape, device="cuda")
    for n in range(3):
        S_chai = to_np(sim.strain(capi.LBM_STRAIN_CHAI))
        sim.step(1, S_out=S, strain_kind=capi.LBM_STRAIN_YU)
        Sy, Sc = ref.step(1)
        assert strain_rel_err(to_np(S), Sy) < 1e-4, n
        assert strain_rel_err(S_chai, Sc) < 1e-4, n
        assert _pop_err(to_np(sim.populations()), ref.g) < 1e-5, n
    Sy = ref.strain("yu")
    ss = float((Sy[0] ** 2 + Sy[1] ** 2 + 2 * Sy[2] ** 2).sum())
    assert abs(sim.reduce()["ss"] - ss) < 1e-4 * ss


def test_taylor_green_64_squared_800_steps():
    """Rotated Taylor-Green vortex on D2Q9, 64^2, diffusive-scaling parameters of the
    convergence study (u0 = 0.025, 800 steps): strain every 100 steps against the oracle
    and S_xy against the closed form."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    N, tau, u0, steps = 64, 0.8, 0.025, 800
    shape = (1, N, N)
    dr, u, gu = synth.tgv_rotated(shape, u0, 1.0)
    op, cp = _spec(shape, tau=tau)
    sim = lbm.LBM(cp, lbm.rho_u_field(dr, u[:2]), lbm.grad_field(gu))
    ref = od.Simulation(op, od.init_populations(dr, u[:2], op, gu[:2, :2]))
    for _ in range(8):
        sim.step(100)
        ref.step(100)
        for kind, okind in ((capi.LBM_STRAIN_YU, "yu"), (capi.LBM_STRAIN_CHAI, "chai")):
            assert strain_rel_err(to_np(sim.strain(kind)), ref.strain(okind)) < 1e-4
    assert _pop_err(to_np(sim.populations()), ref.g) < 1e-5
    exact = cf.tgv_rotated_strain(shape, u0, cf.nu_of_rate(1 / tau), steps)[3]
    S = to_np(sim.strain(capi.LBM_STRAIN_YU))[2]
    assert np.linalg.norm(S - exact) / np.linalg.norm(exact) < 2e-3
    d = sim.reduce()
    assert d["nonfinite"] == 0 and abs(d["mass"] - dr.sum()) < 1e-4 * np.abs(dr).sum()


@pytest.mark.slow
def test_les_4096_squared_sampled():
    """The D2Q9 workload bench.py times (4096^2, FP32, Smagorinsky C_s = 0.1 from the Yu-type
    strain, tau_nu0 = 0.51), in that launch configuration: 16 steps, then populations and
    the strain of every step at sampled nodes against the FP64 oracle run on each node's
    33 x 33 neighbourhood (a node after k steps depends only on its radius-k neighbourhood)."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    from tests._common import sample_nodes
    m, K = 4096, 16
    shape = (1, m, m)
    u = synth.spectrum_velocity(shape, seed=1704, u_rms=0.04)[:2]
    kw = dict(visc="smagorinsky", drive="yu", nu0=(0.51 - 0.5) / 3.0, c_smag=0.1)
    op, cp = _spec(shape, tau=0.51, **kw)
    sim = lbm.LBM(cp, lbm.rho_u_field(np.zeros(shape), u))
    S = [torch.empty((3,) + shape, device="cuda") for _ in range(K)]
    for k in range(K):
        sim.step(1, S_out=S[k], strain_kind=capi.LBM_STRAIN_YU)
    g = sim.populations()
    d = sim.reduce()
    worst_g, dS, fr = 0.0, 0.0, 0.0
    for (_, y, x) in sample_nodes(shape, 30, 9):
        ix = np.ix_([0], [(y + t) % m for t in range(-K, K + 1)], [(x + t) % m for t in range(-K, K + 1)])
        up = np.stack([u[c][ix] for c in range(2)])
        ref = od.Simulation(op, od.init_populations(np.zeros(up.shape[1:]), up, op))
        S_ref = [ref.step(1)[0][:, 0, K, K] for _ in range(K)]
        got = g[:, 0, y, x].double().cpu().numpy()
        worst_g = max(worst_g, _pop_err(got[:, None, None, None], ref.g[:, :, K:K + 1, K:K + 1]))
        for k in range(K):
            dS = max(dS, float(np.abs(S[k][:, 0, y, x].double().cpu().numpy() - S_ref[k]).max()))
            fr = max(fr, float(np.sqrt(S_ref[k][0] ** 2 + S_ref[k][1] ** 2 + 2 * S_ref[k][2] ** 2)))
    sim.close()
    assert worst_g < 1e-5 and dS / fr < 1e-4, (worst_g, dS / fr)
    assert d["nonfinite"] == 0


@pytest.mark.parametrize("shape,walls", [((1, 1, 1), False), ((1, 2, 1), True), ((1, 1, 3), False), ((1, 3, 2), True)])
def test_degenerate_boxes(shape, walls):
    """Boxes one or two nodes wide along some axes (populations wrap onto the node itself or
    its only neighbour): three steps with a force field and lagged Smagorinsky against the
    oracle."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    F = synth.uniform_random_force(shape, seed=21, amp=1e-4)[:2]
    op, cp = _spec(shape, walls=walls, force=F, visc="smagorinsky", drive="chai", nu0=0.01, c_smag=0.3)
    sim = lbm.LBM(cp)
    g0 = synth.random_state(9, shape, seed=22, scale=3e-3).astype(np.float32).astype(np.float64)
    sim.set_populations(torch.as_tensor(g0.astype(np.float32)).cuda())
    ref = od.Simulation(op, g0)
    S = torch.empty((3,) + shape, device="cuda")
    for n in range(3):
        sim.step(1, S_out=S, strain_kind=capi.LBM_STRAIN_CHAI)
        Sy, Sc = ref.step(1)
        assert strain_rel_err(to_np(S), Sc) < 1e-4, n
        assert _pop_err(to_np(sim.populations()), ref.g) < 1e-5, n
    sim.close()
