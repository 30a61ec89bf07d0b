"""Checkpoint / resume and the guarded run loop (paper_1704_07559_amd.checkpoint): host-side
format checks on the CPU, bit-identical resume and rollback on the GPU. Failures are forced
from the host (a NaN written through lbm_set_populations, a tight Mach limit)."""
import numpy as np
import pytest
import torch

import synth
from tests._common import needs_gpu, spec_params


def test_params_roundtrip_through_a_weights_only_file(tmp_path):
    from paper_1704_07559_amd import capi, checkpoint
    p = capi.Params(nx=8, ny=6, nz=4, s=[0.0, 1.19] + [1.25] * 17, visc_kind=capi.LBM_VISC_POWERLAW,
                    K_pl=0.02, n_pl=0.6, walls_y=1, force=(0.0, 0.0, 1e-6))
    f = tmp_path / "p.pt"
    torch.save({"params": checkpoint._params_dict(p), "state": torch.zeros(16, dtype=torch.uint8)}, f)
    d = torch.load(f, weights_only=True)
    q = capi.Params(**d["params"])
    assert q == dataclass_without_field(p)
    e = checkpoint.Diverged(200, "1 non-finite populations", {})
    assert e.step == 200 and "rolled back to step 200" in str(e)


def dataclass_without_field(p):
    import dataclasses
    q = dataclasses.replace(p)
    q.s = [float(v) for v in p.s]
    q.force = [float(v) for v in p.force]
    return q


def _les(shape, seed=5):
    from paper_1704_07559_amd import lbm
    u = synth.spectrum_velocity(shape, seed=1704, u_rms=0.04)
    F = synth.uniform_random_force(shape, seed=seed, amp=1e-5)
    _, cp, _ = spec_params(shape, tau=0.6, visc="smagorinsky", nu0=(0.6 - 0.5) / 3.0, c_smag=0.1, force=F)
    return lbm.LBM(cp, lbm.rho_u_field(np.zeros(shape), u))


@pytest.mark.gpu
@needs_gpu
def test_resume_from_a_file_is_bit_identical(tmp_path):
    from paper_1704_07559_amd import checkpoint
    shape = (16, 24, 32)
    sim = _les(shape)
    sim.step(30)
    checkpoint.save_checkpoint(sim, tmp_path / "c.pt")
    sim.step(20)
    ref, ref_snu = sim.populations(), sim.s_nu.clone()
    sim.close()
    res = checkpoint.load_checkpoint(tmp_path / "c.pt")
    assert res.step_count == 30
    res.step(20)
    assert res.step_count == 50
    assert torch.equal(res.populations(), ref) and torch.equal(res.s_nu, ref_snu)
    res.close()


@pytest.mark.gpu
@needs_gpu
def test_guarded_run_rolls_back_a_non_finite_state():
    from paper_1704_07559_amd import checkpoint
    shape = (16, 24, 32)
    clean = _les(shape)
    clean.step(200)
    ref = clean.populations()
    clean.close()

    def inject(sim, step):
        if step == 300:
            g = sim.populations()
            g[4, 3, 2, 1] = float("nan")
            sim.set_populations(g)

    sim = _les(shape)
    with pytest.raises(checkpoint.Diverged) as e:
        checkpoint.run_guarded(sim, 500, check_every=100, after_chunk=inject)
    assert e.value.step == 200 and "non-finite" in e.value.reason
    assert sim.step_count == 200
    assert torch.equal(sim.populations(), ref)
    d = checkpoint.run_guarded(sim, 100, check_every=50)      # the rolled-back state runs on
    assert d["nonfinite"] == 0 and sim.step_count == 300
    sim.close()


@pytest.mark.gpu
@needs_gpu
def test_guarded_run_mach_watchdog():
    from paper_1704_07559_amd import checkpoint
    sim = _les((8, 8, 64))
    g0 = sim.populations()
    with pytest.raises(checkpoint.Diverged) as e:
        checkpoint.run_guarded(sim, 50, check_every=10, umax_limit=1e-3)
    assert e.value.step == 0 and "max |u|" in e.value.reason
    assert torch.equal(sim.populations(), g0)
    sim.close()
