"""Seeded random configurations of the step on every lattice against the FP64 oracles: box
shapes whose row length picks every launch shape (whole rows with masked lanes, whole rows
through LDS with one to four rows per block, part rows, one node), every viscosity kind and
drive, walls, no / uniform / field forcing, the force-corrected strain, and tau (D3Q19 also
rho0). Three steps from a far-from-equilibrium state each; populations 1e-5 and both strain
formulas 1e-4, as for the fixed cases; the D2Q9 ones again on boxes at least 256 wide, where
steps run two per launch; with 16-bit storage, the bit-exact rounding property of the storage
tests; and one D3Q19 adjoint step per configuration against the oracle's."""
import numpy as np
import pytest

import synth
from tests._common import needs_gpu, pop_rel_err, spec_params, strain_rel_err, to_np

pytestmark = [pytest.mark.gpu, needs_gpu]

NX = [1, 2, 3, 17, 63, 64, 65, 128, 130, 192, 255, 256, 257, 320, 384, 448]
VISC = ["const", "smagorinsky", "powerlaw", "smagorinsky_implicit"]
NCONF = {"d3q19": 24, "d3q15": 12, "d2q9": 12}
CASES = [(lat, k) for lat, n in NCONF.items() for k in range(n)]


def _config(lat, k):
    rng = np.random.default_rng({"d3q19": 1704, "d3q15": 7559, "d2q9": 2017}[lat] + k)
    nx = int(NX[k % len(NX)])
    ny = int(rng.integers(1, 13))
    nz = 1 if lat == "d2q9" else int(rng.integers(1, 5))
    while nx * ny * nz > 24000:
        ny = max(1, ny // 2)
        nz = max(1, nz // 2)
    walls = bool(rng.integers(0, 2)) and ny >= 2
    visc = VISC[int(rng.integers(0, len(VISC)))]
    tau = float(rng.uniform(0.55, 1.2))
    kw = dict(tau=tau, walls=walls, visc=visc, drive=["yu", "chai"][int(rng.integers(0, 2))])
    rho0 = float(rng.choice([1.0, 1.5]))
    if lat == "d3q19":
        kw["rho0"] = rho0
    if visc in ("smagorinsky", "smagorinsky_implicit"):
        kw.update(nu0=(tau - 0.5) / 3.0, c_smag=float(rng.uniform(0.05, 0.5)))
    elif visc == "powerlaw":
        kw.update(K_pl=float(rng.uniform(0.01, 0.3)), n_pl=float(rng.choice([0.5, 0.8, 1.3])), nu_min=1e-3,
                  nu_max=1.0)
    force = ["none", "uniform", "field"][int(rng.integers(0, 3))]
    corrected = force != "none" and bool(rng.integers(0, 2))
    return (nz, ny, nx), kw, force, corrected


def _setup(lat, k):
    shape, kw, force, corrected = _config(lat, k)
    print(f"{lat} config {k}: shape {shape} {kw} force={force} corrected={corrected}", flush=True)
    dim = 2 if lat == "d2q9" else 3
    if force == "uniform":
        kw["force"] = np.array([2e-5, -1e-5, 5e-6][:dim])
    elif force == "field":
        kw["force"] = synth.uniform_random_force(shape, seed=100 + k, amp=1e-4)[:dim]
    if lat == "d3q19":
        from oracle import d3q19 as od
        op, cp, _ = spec_params(shape, **kw)
        q, ncomp, rho0 = 19, 6, kw["rho0"]
    elif lat == "d3q15":
        from oracle import d3q15 as od
        from tests.test_gpu_d3q15 import _spec
        op, cp = _spec(shape, **kw)
        q, ncomp, rho0 = 15, 6, 1.0
    else:
        from oracle import d2q9 as od
        from tests.test_gpu_d2q9 import _spec
        op, cp = _spec(shape, **kw)
        q, ncomp, rho0 = 9, 3, 1.0
    if corrected:
        op.force_corrected = True
        cp.strain_force_correction = 1
    return shape, od, op, cp, q, ncomp, rho0


@pytest.mark.parametrize("lat,k", CASES)
def test_random_configuration(lat, k):
    import torch
    from paper_1704_07559_amd import capi, lbm
    shape, od, op, cp, q, ncomp, rho0 = _setup(lat, k)
    sim = lbm.LBM(cp)
    g0 = synth.random_state(q, shape, seed=200 + k, scale=3e-3).astype(np.float32).astype(np.float64)
    sim.set_populations(torch.as_tensor(g0.astype(np.float32)).cuda())
    ref = od.Simulation(op, g0)
    S = torch.empty((ncomp,) + shape, device="cuda")
    for n in range(3):
        S_chai = to_np(sim.strain(capi.LBM_STRAIN_CHAI))
        sim.step(1, S_out=S, strain_kind=capi.LBM_STRAIN_YU)
        out = ref.step(1)
        Sy, Sc = (out.S_yu, out.S_chai) if lat == "d3q19" else out
        assert strain_rel_err(to_np(S), Sy) < 1e-4, n
        assert strain_rel_err(S_chai, Sc) < 1e-4, n
        assert pop_rel_err(to_np(sim.populations()), ref.g, rho0, od.W) < 1e-5, n
    sim.close()


@pytest.mark.parametrize("k", range(NCONF["d2q9"]))
def test_random_d2q9_configuration_two_steps_per_launch(k):
    """The D2Q9 configurations above on boxes at least 256 wide, where lbm_step takes its steps
    two per launch: eight steps in two groups, with a strain output, against the oracle after
    each group (populations 1e-5; the output, the last step's strain, and both formulas on the
    final state 1e-4)."""
    import torch
    from paper_1704_07559_amd import capi, lbm
    shape, kw, force, corrected = _config("d2q9", k)
    shape = (1, shape[1], 256 + 29 * k)
    print(f"d2q9 config {k} two per launch: shape {shape} {kw} force={force} corrected={corrected}", flush=True)
    if force == "uniform":
        kw["force"] = np.array([2e-5, -1e-5])
    elif force == "field":
        kw["force"] = synth.uniform_random_force(shape, seed=700 + k, amp=1e-4)[:2]
    from oracle import d2q9 as od
    from tests.test_gpu_d2q9 import _spec
    op, cp = _spec(shape, **kw)
    if corrected:
        op.force_corrected = True
        cp.strain_force_correction = 1
    sim = lbm.LBM(cp)
    g0 = synth.random_state(9, shape, seed=800 + k, scale=3e-3).astype(np.float32).astype(np.float64)
    sim.set_populations(torch.as_tensor(g0.astype(np.float32)).cuda())
    ref = od.Simulation(op, g0)
    S = torch.empty((3,) + shape, device="cuda")
    for n in range(2):
        sim.step(4, S_out=S, strain_kind=capi.LBM_STRAIN_CHAI)
        ref.step(3)
        Sy, Sc = ref.step(1)
        assert strain_rel_err(to_np(S), Sc) < 1e-4, n
        assert pop_rel_err(to_np(sim.populations()), ref.g, 1.0, od.W) < 1e-5, n
        assert strain_rel_err(to_np(sim.strain(capi.LBM_STRAIN_YU)), ref.strain("yu")) < 1e-4, n
    sim.close()


ROUNDING_CASES = [(lat, k) for lat in NCONF for k in range(8)]


@pytest.mark.parametrize("lat,k", ROUNDING_CASES)
def test_random_configuration_storage_changes_only_the_rounding(lat, k):
    """The same random configurations with FP16 (even k) or BF16 (odd k) storage: from a
    state representable in the format, each of three steps equals the FP32-stored step
    rounded to nearest even, bit for bit, with the same strain and s_nu."""
    import torch
    from oracle import storage as ost
    from paper_1704_07559_amd import capi, lbm
    storage = "f16" if k % 2 == 0 else "bf16"
    shape, od, op, c32, q, ncomp, rho0 = _setup(lat, k)
    _, _, _, cst, _, _, _ = _setup(lat, k)
    cst.storage = {"f16": capi.LBM_F16, "bf16": capi.LBM_BF16}[storage]
    a, b = lbm.LBM(c32), lbm.LBM(cst)
    g0 = ost.round_storage(synth.random_state(q, shape, seed=300 + k, scale=3e-3), storage)
    b.set_populations(torch.as_tensor(g0).cuda())
    Sa, Sb = torch.empty((ncomp,) + shape, device="cuda"), torch.empty((ncomp,) + shape, device="cuda")
    for n in range(3):
        a.set_populations(b.populations())
        if a.s_nu is not None:
            a.s_nu.copy_(b.s_nu)
        a.step(1, S_out=Sa, strain_kind=capi.LBM_STRAIN_CHAI)
        b.step(1, S_out=Sb, strain_kind=capi.LBM_STRAIN_CHAI)
        assert torch.equal(Sa, Sb), n
        got = b.populations().cpu().numpy()
        ref = ost.round_storage(a.populations().cpu().numpy(), storage)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (n, int((got != ref).sum()))
        if a.s_nu is not None:
            assert torch.equal(a.s_nu, b.s_nu), n
    a.close()
    b.close()


def _rel(a, b):
    return float(np.abs(np.asarray(a, dtype=np.float64) - b).max() / np.abs(b).max())


@pytest.mark.parametrize("k", range(NCONF["d3q19"]))
def test_random_configuration_adjoint_step(k):
    """One D3Q19 adjoint step (lbm_adjoint_step) in every D3Q19 configuration above,
    against the oracle's adjoint: dJ/dg, dJ/dF and, for the lagged viscosities, the adjoint
    of the s_nu field; 1e-5 of the largest value, as for the fixed cases."""
    import torch
    from oracle import adjoint as adj
    from oracle import adjoint_visc as av
    from oracle import d3q19 as od
    from paper_1704_07559_amd import capi, lbm
    shape, _, op, cp, _, _, _ = _setup("d3q19", k)
    N = cp.N
    F = op.force
    if F is None:
        F = np.zeros((3,) + shape)
    elif np.asarray(F).shape == (3,):
        F = np.broadcast_to(np.asarray(F, dtype=np.float64).reshape(3, 1, 1, 1), (3,) + shape).copy()
    F = np.asarray(F, dtype=np.float32).astype(np.float64)
    u = synth.random_vector(shape, seed=400 + k, scale=0.05)
    g = od.init_populations(np.zeros(shape), u, op) + synth.random_state(19, shape, seed=500 + k, scale=3e-3)
    g = g.astype(np.float32).astype(np.float64)
    sim = lbm.LBM(cp)
    sim.set_populations(torch.as_tensor(g.astype(np.float32)).cuda())
    sp = None
    if op.visc_kind in ("smagorinsky", "powerlaw"):
        sp = 1.0 / (3.0 * (0.02 + 0.01 * synth.random_state(1, shape, seed=600 + k, scale=1.0)[0] ** 2) + 0.5)
        sp = sp.astype(np.float32).astype(np.float64)
        sim.s_nu.copy_(torch.as_tensor(sp.reshape(-1).astype(np.float32)))
    A = sim.adjoint_planes
    rec = torch.empty((1, sim.save_planes, N), device="cuda")
    sim.step(1, save=rec)
    lam_in = synth.random_state(A, shape, seed=700 + k, scale=1.0).astype(np.float32).astype(np.float64)
    lam_t = torch.as_tensor(lam_in.astype(np.float32)).cuda().reshape(A, N).contiguous()
    lam_out = torch.empty_like(lam_t)
    gF = torch.zeros((3, N), device="cuda")
    capi.lbm_adjoint_step(sim.ctx, rec[0], lam_t, lam_out, gF)
    pf = adj._with_force(op, F)
    out = to_np(lam_out).reshape((A,) + shape)
    if op.visc_kind == "const":
        ref_lam, ref_gF = adj.adjoint_step(lam_in, g, F, pf)
        ref_lams = None
    else:
        ref_lam, ref_lams, ref_gF = av.adjoint_step_visc(lam_in[:19], lam_in[19] if sp is not None else None, g, sp,
                                                         F, pf)
    assert _rel(out[:19], ref_lam) < 1e-5
    if np.abs(ref_gF).max() > 0:
        assert _rel(to_np(gF).reshape(ref_gF.shape), ref_gF) < 1e-5
    if sp is not None:
        assert _rel(out[19], ref_lams) < 1e-5
    sim.close()
