"""Parity of the force-corrected strain (strain_force_correction = 1) with the FP64 oracle on
D3Q19, D3Q15 and D2Q9.

The force here is large (field amplitude 1e-2 against a random state of amplitude 3e-3), so
the correction changes the strain by far more than the 1e-4 parity tolerance; each case
checks that the uncorrected oracle strain is out of tolerance.
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


def test_adjoint_is_rejected_with_the_correction():
    import torch
    from paper_1704_07559_amd import capi, lbm
    shape = (4, 6, 8)
    op, cp, _ = spec_params(shape, force=np.array([1e-4, 0.0, 0.0]))
    cp.strain_force_correction = 1
    sim = lbm.LBM(cp)
    assert capi.lbm_save_planes(sim.ctx) == 0 and capi.lbm_adjoint_planes(sim.ctx) == 0
    rec = torch.empty(3 * 4 * 6 * 8, device="cuda")
    with pytest.raises(capi.LBMError) as e:
        sim.step(1, save=rec)
    assert e.value.status == capi.LBM_EUNSUPPORTED
    sim.close()
