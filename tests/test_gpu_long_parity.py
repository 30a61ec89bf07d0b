"""200-step element-wise parity of the D3Q19 step in the launch shapes the benchmark times.

The benchmark credits three instances of the fused step: whole 256-node rows in one block
with the x-shifted populations exchanged through LDS (the 256^3 LES), whole 128-node rows
with y-walls (the 128 x 128 x 512 channel), and 128-node segments of 384-node rows (the
384^3 runs, 128 x 2 blocks in FP32 and 128 x 1 in FP16/BF16). Each is run here for 200 steps
against the FP64 oracle on a box with the same row length (so the same block shape and the
same kernel instance), with the workload's own parameters:

* LES: lagged Smagorinsky (C_s = 0.1, nu0 = 1/300) driven by the Yu strain, the seeded
  k^4 exp(-2 (k/4)^2) velocity field;
* channel: the same LES parameters with walls and a body force, and the power-law case
  (n = 0.5, Chai drive) of the channel workload.

Populations (relative on f = g + w rho0) and the lagged s_nu field are compared at every
10th step within 1e-5, the emitted strain at every step within 1e-4 of the largest strain
norm of the run (the runs start from the equilibrium, whose strain is zero: the first
snapshots have no scale of their own). The strain is emitted by a runtime switch of the same
kernel; a second run without it must reach the same bits, so the checked trajectory is the
timed one.

With 16-bit storage the arithmetic is FP32 and only the stored deviations are rounded: at
every one of 200 steps the FP16 (BF16) step from its own state equals the FP32 step from the
same state rounded to nearest even, bit for bit, with the same strain and s_nu bits.
"""
import numpy as np
import pytest

import synth
from oracle import d3q19 as od
from tests._common import needs_gpu, pop_rel_err, spec_params, to_np

pytestmark = [pytest.mark.gpu, needs_gpu]

STEPS = 200
LES = dict(tau=0.51, visc="smagorinsky", drive="yu", nu0=(0.51 - 0.5) / 3.0, c_smag=0.1)
POWERLAW = dict(tau=0.8, visc="powerlaw", drive="chai", K_pl=0.1 * (1e-5 * 8 / 0.2) ** 0.5, n_pl=0.5,
                nu_min=1e-3, nu_max=1.0)

# (nz, ny, nx): the row length fixes the block (256 x 1, 128 x 2, 128 x 2 part rows)
CASES = {
    "les_rows256_lds": ((4, 4, 256), LES, False, None),
    "les_channel_rows128_lds": ((4, 8, 128), LES, True, (0.0, 0.0, 1e-5)),
    "powerlaw_channel_rows128_lds": ((4, 8, 128), POWERLAW, True, (0.0, 0.0, 1e-5)),
    "les_part_rows384": ((3, 4, 384), LES, False, None),
}


def _emit_kind(kw):
    from paper_1704_07559_amd import capi
    return capi.LBM_STRAIN_CHAI if kw.get("drive") == "chai" else capi.LBM_STRAIN_YU


@pytest.mark.slow
@pytest.mark.parametrize("case", sorted(CASES))
def test_200_steps_against_oracle(case):
    import torch
    from paper_1704_07559_amd import lbm
    shape, kw, walls, force = CASES[case]
    u = synth.spectrum_velocity(shape, seed=1704, u_rms=0.04)
    F = None if force is None else np.array(force)
    op, cp, _ = spec_params(shape, walls=walls, force=F, **kw)
    ref = od.Simulation(op, od.init_populations(np.zeros(shape), u, op))
    sim = lbm.LBM(cp, lbm.rho_u_field(np.zeros(shape), u))
    quiet = lbm.LBM(cp, lbm.rho_u_field(np.zeros(shape), u))
    kind = _emit_kind(kw)
    S = torch.empty((6,) + shape, device="cuda")
    worst = {"pop": 0.0, "strain": 0.0, "snu": 0.0}
    dS, scale = 0.0, 0.0
    wts = np.array([1, 1, 1, 2, 2, 2], dtype=np.float64).reshape(6, 1, 1, 1)
    for n in range(1, STEPS + 1):
        sim.step(1, S_out=S, strain_kind=kind)
        out = ref.step(1)
        S_ref = out.S_chai if kind == 2 else out.S_yu
        dS = max(dS, float(np.abs(to_np(S) - S_ref).max()))
        scale = max(scale, float(np.sqrt((wts * S_ref**2).sum(axis=0)).max()))
        if n % 10 == 0:
            worst["pop"] = max(worst["pop"], pop_rel_err(to_np(sim.populations()), ref.g, op.rho0))
            snu = to_np(sim.s_nu).reshape(shape)
            worst["snu"] = max(worst["snu"], float(np.abs(snu - ref.s_nu).max() / np.abs(ref.s_nu).max()))
    worst["strain"] = dS / scale
    quiet.step(STEPS)
    same = torch.equal(quiet.populations(), sim.populations()) and torch.equal(quiet.s_nu, sim.s_nu)
    sim.close()
    quiet.close()
    assert worst["pop"] < 1e-5 and worst["strain"] < 1e-4 and worst["snu"] < 1e-5, worst
    assert same


@pytest.mark.slow
@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_200_steps_half_storage_is_the_rounded_fp32_step(storage):
    import torch
    from oracle import storage as ost
    from paper_1704_07559_amd import capi, lbm
    shape = (3, 4, 384)   # 128-node row segments, 128 x 1 blocks with 16-bit storage
    u = synth.spectrum_velocity(shape, seed=1704, u_rms=0.04)
    _, c32, _ = spec_params(shape, **LES)
    _, cst, _ = spec_params(shape, storage=storage, **LES)
    a, b = lbm.LBM(c32), lbm.LBM(cst, lbm.rho_u_field(np.zeros(shape), u))
    Sa, Sb = torch.empty((6,) + shape, device="cuda"), torch.empty((6,) + shape, device="cuda")
    for n in range(STEPS):
        a.set_populations(b.populations())
        a.s_nu.copy_(b.s_nu)
        a.step(1, S_out=Sa, strain_kind=capi.LBM_STRAIN_YU)
        b.step(1, S_out=Sb, strain_kind=capi.LBM_STRAIN_YU)
        assert torch.equal(Sa, Sb), n
        assert torch.equal(a.s_nu, b.s_nu), n
        got = b.populations().cpu().numpy()
        want = ost.round_storage(a.populations().cpu().numpy(), storage)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (n, int((got != want).sum()))
    # the run went somewhere: the state is not the initial one
    assert float(Sb.abs().max()) > 0.0
    a.close()
    b.close()


# The D3Q15 and D2Q9 LES workloads: whole 256-node rows through LDS (D3Q15 at 256^3) and
# 256-node segments of longer rows (D2Q9 at 4096^2, pull mode 0), 200 steps each.
OTHER = {
    "d3q15_les_rows256_lds": ("d3q15", (4, 4, 256)),
    "d2q9_les_part_rows": ("d2q9", (1, 8, 512)),
}


@pytest.mark.slow
@pytest.mark.parametrize("case", sorted(OTHER))
def test_200_steps_other_lattices_against_oracle(case):
    from paper_1704_07559_amd import capi, lbm
    lattice, shape = OTHER[case]
    if lattice == "d3q15":
        from oracle import d3q15 as om
        from tests.test_gpu_d3q15 import _spec
        u = synth.spectrum_velocity(shape, seed=1704, u_rms=0.04)
        ncomp, wts = 6, np.array([1, 1, 1, 2, 2, 2], dtype=np.float64)
    else:
        from oracle import d2q9 as om
        from tests.test_gpu_d2q9 import _spec
        u = synth.spectrum_velocity(shape, seed=1704, u_rms=0.04)[:2]
        ncomp, wts = 3, np.array([1, 1, 2], dtype=np.float64)
    import torch
    op, cp = _spec(shape, tau=0.51, visc="smagorinsky", drive="yu", nu0=(0.51 - 0.5) / 3.0, c_smag=0.1)
    ref = om.Simulation(op, om.init_populations(np.zeros(shape), u, op))
    sim = lbm.LBM(cp, lbm.rho_u_field(np.zeros(shape), u))
    S = torch.empty((ncomp,) + shape, device="cuda")
    wts = wts.reshape((ncomp,) + (1,) * len(shape))
    dS, scale, worst_pop, worst_snu = 0.0, 0.0, 0.0, 0.0
    for n in range(1, STEPS + 1):
        sim.step(1, S_out=S, strain_kind=capi.LBM_STRAIN_YU)
        S_ref = ref.step(1)[0]
        dS = max(dS, float(np.abs(to_np(S) - S_ref).max()))
        scale = max(scale, float(np.sqrt((wts * S_ref**2).sum(axis=0)).max()))
        if n % 10 == 0:
            worst_pop = max(worst_pop, pop_rel_err(to_np(sim.populations()), ref.g, op.rho0, om.W))
            snu = to_np(sim.s_nu).reshape(shape)
            worst_snu = max(worst_snu, float(np.abs(snu - ref.s_nu).max() / np.abs(ref.s_nu).max()))
    sim.close()
    assert worst_pop < 1e-5 and dS / scale < 1e-4 and worst_snu < 1e-5, (worst_pop, dS / scale, worst_snu)
