"""D2Q9 steps taken two per launch (lbm_step on boxes at least 256 wide, periodic or with walls
in y, in groups of four steps) against the same steps taken one launch each, bit for bit:
populations, the lagged s_nu field and the step counter, in every storage type, viscosity law
and force mode, on boxes whose width leaves a ragged last strip and whose height leaves a ragged
last block of rows; then against the FP64 oracle, and replayed from a HIP graph."""
import numpy as np
import pytest

import synth
from oracle import d2q9 as od
from tests._common import needs_gpu, strain_rel_err, to_np
from tests.test_gpu_d2q9 import _pop_err, _spec

pytestmark = [pytest.mark.gpu, needs_gpu]

CASES = {
    "const": dict(),
    "const_uniform_force": dict(force=np.array([2e-5, -1e-5])),
    "smag_yu": dict(visc="smagorinsky", drive="yu", nu0=0.01, c_smag=0.2),
    "smag_yu_force_field": dict(visc="smagorinsky", drive="yu", nu0=0.01, c_smag=0.2, force="field"),
    "powerlaw_chai": dict(visc="powerlaw", drive="chai", K_pl=0.02, n_pl=0.6),
    "smag_implicit_chai": dict(visc="smagorinsky_implicit", drive="chai", nu0=0.005, c_smag=0.2),
    "walls_smag_yu_force": dict(visc="smagorinsky", drive="yu", nu0=0.01, c_smag=0.2, walls=True,
                                force=np.array([2e-5, 0.0])),
    "walls_powerlaw_chai_force_field": dict(visc="powerlaw", drive="chai", K_pl=0.02, n_pl=0.6, walls=True,
                                            force="field"),
    "walls_implicit_yu": dict(visc="smagorinsky_implicit", drive="yu", nu0=0.005, c_smag=0.2, walls=True),
    "corrected_smag_chai_force_field": dict(visc="smagorinsky", drive="chai", nu0=0.01, c_smag=0.2,
                                            force="field", strain_force_correction=1),
    "walls_corrected_implicit_yu_force": dict(visc="smagorinsky_implicit", drive="yu", nu0=0.005, c_smag=0.2,
                                              walls=True, force=np.array([2e-5, 0.0]), strain_force_correction=1),
}


def _pair(shape, case, storage, seed):
    """Two contexts on the same random state: one to be stepped in groups, one singly."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    kw = dict(CASES[case])
    corr = kw.pop("strain_force_correction", 0)
    if isinstance(kw.get("force"), str):
        kw["force"] = synth.uniform_random_force(shape, seed=seed + 1, amp=1e-4)[:2]
    _, cp = _spec(shape, **kw)
    cp.storage = storage
    cp.strain_force_correction = corr
    g0 = torch.as_tensor(synth.random_state(9, shape, seed=seed, scale=3e-3).astype(np.float32)).cuda()
    sims = []
    for _ in range(2):
        sim = lbm.LBM(cp)
        sim.set_populations(g0)
        sims.append(sim)
    if cp.visc_kind in (capi.LBM_VISC_SMAGORINSKY, capi.LBM_VISC_POWERLAW):
        # a non-uniform lagged field, as after a first step
        sims[0].step(1)
        sims[1].step(1)
    return sims


def _assert_same(a, b, msg):
    import torch
    torch.cuda.synchronize()
    assert torch.equal(a.populations(), b.populations()), msg
    if a.s_nu is not None:
        assert torch.equal(a.s_nu, b.s_nu), msg
    assert a.step_count == b.step_count, msg


@pytest.mark.parametrize("shape", [(1, 37, 256), (1, 35, 509), (1, 3, 600), (1, 18, 4096)])
@pytest.mark.parametrize("case", sorted(CASES))
def test_grouped_steps_equal_single_steps(case, shape):
    from paper_1704_07559_amd import capi
    grouped, single = _pair(shape, case, capi.LBM_F32, seed=31)
    for n in (4, 5, 7, 10):                     # groups of four, and 1, 3 or 2 single steps after them
        grouped.step(n)
        for _ in range(n):
            single.step(1)
        _assert_same(grouped, single, (case, shape, n))
    grouped.close()
    single.close()


@pytest.mark.parametrize("shape,walls", [((1, 1, 256), False), ((1, 2, 300), False), ((1, 2, 300), True),
                                         ((1, 7, 257), False), ((1, 7, 257), True)])
def test_grouped_steps_on_degenerate_heights(shape, walls):
    """Boxes one to a few rows high (rows wrap onto themselves, or the two walls bound two rows)
    and a strip of one column past the first: grouped steps against single steps, bit for bit."""
    from paper_1704_07559_amd import capi
    case = "walls_smag_yu_force" if walls else "smag_yu_force_field"
    grouped, single = _pair(shape, case, capi.LBM_F32, seed=81)
    grouped.step(8)
    for _ in range(8):
        single.step(1)
    _assert_same(grouped, single, (shape, walls))
    grouped.close()
    single.close()


@pytest.mark.parametrize("kind", ["yu", "chai"])
@pytest.mark.parametrize("case", ["smag_yu", "walls_implicit_yu", "smag_yu_force_field",
                                  "corrected_smag_chai_force_field"])
def test_grouped_steps_with_strain_output(case, kind):
    """With a strain output the launches of two steps write the second step's strain, which is
    what single steps leave there last: after 4, 5 and 10 steps the output holds the same bits."""
    import torch
    from paper_1704_07559_amd import capi
    shape = (1, 35, 509)
    sk = {"yu": capi.LBM_STRAIN_YU, "chai": capi.LBM_STRAIN_CHAI}[kind]
    grouped, single = _pair(shape, case, capi.LBM_F32, seed=71)
    Sg = torch.full((3,) + shape, float("nan"), device="cuda")
    Ss = torch.full((3,) + shape, float("nan"), device="cuda")
    for n in (4, 5, 10):
        grouped.step(n, S_out=Sg, strain_kind=sk)
        for _ in range(n):
            single.step(1, S_out=Ss, strain_kind=sk)
        _assert_same(grouped, single, (case, kind, n))
        torch.cuda.synchronize()
        assert torch.equal(Sg, Ss), (case, kind, n)
    grouped.close()
    single.close()


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("case", ["smag_yu", "smag_yu_force_field", "smag_implicit_chai", "walls_smag_yu_force"])
def test_grouped_steps_equal_single_steps_16_bit(case, storage):
    """16-bit storage: the intermediate level is rounded as a store would round it."""
    from paper_1704_07559_amd import capi
    st = {"f16": capi.LBM_F16, "bf16": capi.LBM_BF16}[storage]
    grouped, single = _pair((1, 35, 509), case, st, seed=41)
    grouped.step(8)
    for _ in range(8):
        single.step(1)
    _assert_same(grouped, single, (case, storage))
    grouped.close()
    single.close()


def test_grouped_steps_against_oracle():
    """Twelve steps in three groups from a far-from-equilibrium state with a force field and
    lagged Smagorinsky: populations and both strains against the FP64 oracle."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    shape = (1, 33, 300)
    F = synth.uniform_random_force(shape, seed=52, amp=1e-4)[:2]
    op, cp = _spec(shape, visc="smagorinsky", drive="yu", nu0=0.01, c_smag=0.2, force=F)
    sim = lbm.LBM(cp)
    g0 = synth.random_state(9, shape, seed=53, scale=3e-3).astype(np.float32).astype(np.float64)
    sim.set_populations(torch.as_tensor(g0.astype(np.float32)).cuda())
    ref = od.Simulation(op, g0)
    for _ in range(3):
        sim.step(4)
        ref.step(4)
        assert _pop_err(to_np(sim.populations()), ref.g) < 1e-5
        for kind, okind in ((capi.LBM_STRAIN_YU, "yu"), (capi.LBM_STRAIN_CHAI, "chai")):
            assert strain_rel_err(to_np(sim.strain(kind)), ref.strain(okind)) < 1e-4
    assert sim.step_count == 12
    sim.close()


def test_grouped_steps_with_walls_against_oracle():
    """A channel between halfway bounce-back walls in y, driven by a uniform force, with lagged
    Smagorinsky from the Chai strain: twelve steps in three groups from a far-from-equilibrium
    state against the FP64 oracle (the rows next to the walls take their crossing populations
    from the node's own intermediate state)."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    shape = (1, 29, 300)
    op, cp = _spec(shape, visc="smagorinsky", drive="chai", nu0=0.01, c_smag=0.2, walls=True,
                   force=np.array([1e-5, 0.0]))
    sim = lbm.LBM(cp)
    g0 = synth.random_state(9, shape, seed=54, scale=3e-3).astype(np.float32).astype(np.float64)
    sim.set_populations(torch.as_tensor(g0.astype(np.float32)).cuda())
    ref = od.Simulation(op, g0)
    for _ in range(3):
        sim.step(4)
        ref.step(4)
        assert _pop_err(to_np(sim.populations()), ref.g) < 1e-5
        for kind, okind in ((capi.LBM_STRAIN_YU, "yu"), (capi.LBM_STRAIN_CHAI, "chai")):
            assert strain_rel_err(to_np(sim.strain(kind)), ref.strain(okind)) < 1e-4
    sim.close()


def test_grouped_steps_captured_in_a_graph_replay_exactly():
    """Four steps (two launches of two) captured into a HIP graph: every replay gives the bits
    of four eager single steps, with eager work between the replays."""
    import torch
    from paper_1704_07559_amd import capi
    cap, eager = _pair((1, 20, 512), "smag_yu", capi.LBM_F32, seed=61)
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        with torch.cuda.graph(graph, stream=st):
            cap.step(4)
    torch.cuda.synchronize()
    for rep in range(3):
        graph.replay()
        for _ in range(4):
            eager.step(1)
        torch.cuda.synchronize()
        assert torch.equal(cap.populations(), eager.populations()), rep
        assert torch.equal(cap.s_nu, eager.s_nu), rep
        assert cap.reduce()["nonfinite"] == 0
    cap.close()
    eager.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_les_4096_squared_grouped_equal_single(storage):
    """The D2Q9 workload bench.py times (4096^2, lagged Smagorinsky C_s = 0.1 from the Yu-type
    strain, tau_nu0 = 0.51, spectrum velocity), in FP32 and FP16 storage: 16 steps in four
    groups against 16 single steps, bit for bit."""
    from paper_1704_07559_amd import capi, lbm
    m = 4096
    shape = (1, m, m)
    u = synth.spectrum_velocity(shape, seed=1704, u_rms=0.04)[:2]
    _, cp = _spec(shape, tau=0.51, visc="smagorinsky", drive="yu", nu0=(0.51 - 0.5) / 3.0, c_smag=0.1)
    cp.storage = {"f32": capi.LBM_F32, "f16": capi.LBM_F16}[storage]
    rho_u = lbm.rho_u_field(np.zeros(shape), u)
    grouped, single = lbm.LBM(cp, rho_u), lbm.LBM(cp, rho_u)
    grouped.step(16)
    for _ in range(16):
        single.step(1)
    _assert_same(grouped, single, "4096^2")
    assert grouped.reduce()["nonfinite"] == 0
    grouped.close()
    single.close()


def test_les_4096_squared_grouped_sampled_against_oracle():
    """The D2Q9 workload in the launch configuration bench.py times (4096^2 FP32, lagged
    Smagorinsky from the Yu-type strain, two steps per launch): 16 steps in four groups with a
    strain output, then the populations and the last step's strain at sampled nodes (the box's
    corners among them) against the FP64 oracle run on each node's 33 x 33 neighbourhood."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    from tests._common import sample_nodes
    m, K = 4096, 16
    shape = (1, m, m)
    u = synth.spectrum_velocity(shape, seed=1704, u_rms=0.04)[:2]
    op, cp = _spec(shape, tau=0.51, visc="smagorinsky", drive="yu", nu0=(0.51 - 0.5) / 3.0, c_smag=0.1)
    sim = lbm.LBM(cp, lbm.rho_u_field(np.zeros(shape), u))
    S = torch.empty((3,) + shape, device="cuda")
    sim.step(K, S_out=S, strain_kind=capi.LBM_STRAIN_YU)
    g = sim.populations()
    worst_g, dS, fr = 0.0, 0.0, 0.0
    for (_, y, x) in sample_nodes(shape, 24, 19):
        ix = np.ix_([0], [(y + t) % m for t in range(-K, K + 1)], [(x + t) % m for t in range(-K, K + 1)])
        up = np.stack([u[c][ix] for c in range(2)])
        ref = od.Simulation(op, od.init_populations(np.zeros(up.shape[1:]), up, op))
        for _ in range(K - 1):
            ref.step(1)
        S_ref = ref.step(1)[0][:, 0, K, K]
        got = g[:, 0, y, x].double().cpu().numpy()
        worst_g = max(worst_g, _pop_err(got[:, None, None, None], ref.g[:, :, K:K + 1, K:K + 1]))
        dS = max(dS, float(np.abs(S[:, 0, y, x].double().cpu().numpy() - S_ref).max()))
        fr = max(fr, float(np.sqrt(S_ref[0] ** 2 + S_ref[1] ** 2 + 2 * S_ref[2] ** 2)))
    sim.close()
    assert worst_g < 1e-5 and dS / fr < 1e-4, (worst_g, dS / fr)

