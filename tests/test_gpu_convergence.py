"""Second-order spatial accuracy of the strain on the GPU (Section 5.1: the strain of either
formula is second-order accurate). Rotated Taylor-Green vortex in the xy plane under diffusive
scaling (u0 ~ 1/N, steps ~ N^2), the FP32 library run from the Chapman-Enskog initial state,
S_xy against the closed form of oracle/closed_forms.py at equal physical time, N = 16, 32, 64
(the ladder the FP64 oracle is pinned on). Both formulas: Yu from the step's strain output,
Chai from the strain query. The GPU error also equals the FP64 oracle's on the same flow, so
what is measured is the method's discretisation error, not FP32 round-off."""
import numpy as np
import pytest

import synth
from oracle import closed_forms as cf
from oracle import d3q19 as od
from tests._common import needs_gpu, spec_params

pytestmark = [pytest.mark.gpu, needs_gpu]

TAU = 0.8


def _setup(N):
    u0 = 0.05 * 32 / N
    steps = int(round(200 * (N / 32) ** 2))
    shape = (1, N, N)
    return u0, steps, shape


def _gpu_errors(N):
    """Relative L2 error of S_xy: (Yu at level steps - 1, Chai at level steps + 1)."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    u0, steps, shape = _setup(N)
    _, cp, _ = spec_params(shape, tau=TAU)
    dr, u, gu = synth.tgv_rotated(shape, u0, 1.0, (0, 1))
    sim = lbm.LBM(cp, lbm.rho_u_field(dr, u), lbm.grad_field(gu))
    S = torch.empty((6,) + shape, device="cuda")
    sim.step(steps, S_out=S, strain_kind=capi.LBM_STRAIN_YU)  # strain of the state at steps - 1
    sim.step(1)
    chai = sim.strain(capi.LBM_STRAIN_CHAI).double().cpu().numpy()
    yu = S.double().cpu().numpy()
    sim.close()
    nu = cf.nu_of_rate(1.0 / TAU)
    ex_yu = cf.tgv_rotated_strain(shape, u0, nu, steps - 1, (0, 1))
    ex_chai = cf.tgv_rotated_strain(shape, u0, nu, steps + 1, (0, 1))
    rel = lambda a, b: float(np.linalg.norm(a[3] - b[3]) / np.linalg.norm(b[3]))
    return rel(yu, ex_yu), rel(chai, ex_chai)


def test_strain_converges_at_second_order_fp32():
    errs = np.array([_gpu_errors(N) for N in (16, 32, 64)])  # columns: Yu, Chai
    orders = np.log2(errs[:-1] / errs[1:])
    assert (orders >= 1.8).all(), (errs.tolist(), orders.tolist())
    assert errs[-1].max() < 1e-3, errs.tolist()


@pytest.mark.parametrize("N", [16, 64])
def test_gpu_error_equals_the_oracle_error(N):
    """The same rung run by the FP64 oracle: the two discretisation errors agree to 1e-3 of
    their size (at N = 64, 800 steps, they differ in the fifth digit)."""
    u0, steps, shape = _setup(N)
    p = od.Params(s=od.default_rates(TAU))
    dr, u, gu = synth.tgv_rotated(shape, u0, 1.0, (0, 1))
    ref = od.Simulation(p, od.init_populations(dr, u, p, gu))
    ref.step(steps + 1)
    ex = cf.tgv_rotated_strain(shape, u0, cf.nu_of_rate(1.0 / TAU), steps + 1, (0, 1))
    e_ref = float(np.linalg.norm(ref.strain("chai")[3] - ex[3]) / np.linalg.norm(ex[3]))
    e_gpu = _gpu_errors(N)[1]
    assert abs(e_gpu - e_ref) <= 1e-3 * e_ref, (e_gpu, e_ref)
