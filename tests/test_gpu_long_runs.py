"""Full-length runs of the benchmarked workloads at their full sizes, checked through
properties that hold at any size and length.

* LES 256^3, FP32, lagged Smagorinsky from the Yu strain, 1000 steps (the headline
  workload): no non-finite population and max |u| under the Mach watchdog (0.4) at every
  100-step check; total mass and momentum (periodic box, no force) constant to 1e-9 of
  N rho0 (the collision conserves both exactly, Eq. continuityandmomentum, so only FP32
  rounding moves them); kinetic energy falling from check to check (an unforced flow with a
  positive eddy viscosity only dissipates); and translation invariance, bit for bit: the
  same run started from the initial field shifted by (5, 3, 1) nodes ends in the shifted
  state (every node computes the same function of its neighbourhood, across block and row
  boundaries alike).
* The channel 128 x 128 x 512 (walls in y, force 1e-6 along z, power law n = 0.5 and 1.5
  driven by the Chai strain), 5000 steps from rest: the flow stays exactly uniform in x and z
  (every row the same bits), so the full run is element by element the 1-D channel, which
  the FP64 oracle runs for the same 5000 steps: populations within 1e-5 (relative on f), the
  velocity profile within 1e-4 of its peak, the Chai strain within 1e-4 of its largest norm,
  the s_nu field within 1e-4; mass constant to 1e-9 of N rho0.
"""
import numpy as np
import pytest

import synth
from oracle import d3q19 as od
from tests._common import needs_gpu, pop_rel_err, spec_params, strain_rel_err

pytestmark = [pytest.mark.gpu, needs_gpu]


@pytest.mark.slow
def test_les_256_cubed_1000_steps():
    import torch
    from paper_1704_07559_amd import lbm
    shape = (256, 256, 256)
    N = 256 ** 3
    shift = (5, 3, 1)
    u = synth.spectrum_velocity(shape, seed=1704, u_rms=0.04)
    _, cp, _ = spec_params(shape, tau=0.51, visc="smagorinsky", drive="yu", nu0=(0.51 - 0.5) / 3.0, c_smag=0.1)
    sim = lbm.LBM(cp, lbm.rho_u_field(np.zeros(shape), u))
    moved = lbm.LBM(cp, lbm.rho_u_field(np.zeros(shape), np.roll(u, shift, axis=(1, 2, 3))))
    del u
    d0 = sim.reduce()
    diags = [d0]
    for _ in range(10):
        sim.step(100)
        moved.step(100)
        diags.append(sim.reduce())
    same = torch.equal(moved.populations(), torch.roll(sim.populations(), shift, dims=(1, 2, 3)))
    same_snu = torch.equal(moved.s_nu.reshape(shape), torch.roll(sim.s_nu.reshape(shape), shift, dims=(0, 1, 2)))
    sim.close()
    moved.close()
    for k, d in enumerate(diags):
        assert d["nonfinite"] == 0, k
        assert d["umax"] < 0.4, (k, d["umax"])
    assert abs(diags[-1]["mass"] - d0["mass"]) < 1e-9 * N * cp.rho0, [d["mass"] for d in diags]
    assert np.abs(diags[-1]["mom"] - d0["mom"]).max() < 1e-9 * N * cp.rho0, [list(d["mom"]) for d in diags]
    ke = [d["ke"] for d in diags]
    assert all(b < a for a, b in zip(ke[:-1], ke[1:])), ke
    assert ke[-1] < 0.9 * ke[0], ke
    assert same and same_snu


@pytest.mark.slow
@pytest.mark.parametrize("n_pl", [0.5, 1.5])
def test_powerlaw_channel_5000_steps_is_the_1d_channel(n_pl):
    import torch
    from paper_1704_07559_amd import capi, lbm
    shape = (512, 128, 128)   # (nz, ny, nx)
    N = 512 * 128 * 128
    Fz = 1e-6
    steps = 5000
    gref = Fz * 128 / (2 * 0.1)   # wall shear rate of the Newtonian flow with nu = 0.1
    kw = dict(tau=0.8, visc="powerlaw", drive="chai", K_pl=0.1 * gref ** (1 - n_pl), n_pl=n_pl, nu_min=1e-3,
              nu_max=1.0, walls=True, force=np.array([0.0, 0.0, Fz]))
    _, cp, _ = spec_params(shape, **kw)
    sim = lbm.LBM(cp)
    d0 = sim.reduce()
    sim.step(steps)
    d1 = sim.reduce()
    g = sim.populations()                                   # (19, nz, ny, nx)
    uniform = bool(torch.equal(g, g[:, :1, :, :1].expand_as(g)))
    prof = g[:, 0, :, 0].double().cpu().numpy()             # (19, ny)
    snu = sim.s_nu.reshape(shape)
    snu_uniform = bool(torch.equal(snu, snu[:1, :, :1].expand_as(snu)))
    snu_prof = snu[0, :, 0].double().cpu().numpy()
    S = sim.strain(capi.LBM_STRAIN_CHAI)[:, 0, :, 0].double().cpu().numpy()
    sim.close()
    del g

    shape1 = (1, 128, 1)
    op, _, _ = spec_params(shape1, **kw)
    ref = od.Simulation(op, od.init_populations(np.zeros(shape1), np.zeros((3,) + shape1), op))
    ref.step(steps)
    g_ref = ref.g[:, 0, :, 0]
    S_ref = ref.strain("chai")[:, 0, :, 0]
    uz = (od.C[2].astype(np.float64) @ prof + 0.5 * Fz) / op.rho0
    uz_ref = (od.C[2].astype(np.float64) @ g_ref + 0.5 * Fz) / op.rho0

    assert uniform and snu_uniform
    assert d0["nonfinite"] == 0 and d1["nonfinite"] == 0
    assert abs(d1["mass"] - d0["mass"]) < 1e-9 * N * cp.rho0, (d0["mass"], d1["mass"])
    assert pop_rel_err(prof, g_ref, op.rho0) < 1e-5
    assert np.abs(uz - uz_ref).max() < 1e-4 * np.abs(uz_ref).max(), np.abs(uz - uz_ref).max() / uz_ref.max()
    assert strain_rel_err(S, S_ref) < 1e-4
    # s_nu follows |S|^(n-1) pointwise; where |S| nears zero (mid-channel, 1e-7) it comes from
    # non-equilibrium moments 1e-3 of the stored deviations, whose FP32 rounding then shows
    # (1.4e-5 measured for n = 1.5): held to the strain's own 1e-4
    assert np.abs(snu_prof - ref.s_nu[0, :, 0]).max() < 1e-4 * ref.s_nu.max()
