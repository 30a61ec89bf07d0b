"""The largest boxes the library accepts: each lattice and storage at the z-plane size limit
of its 32-bit in-plane byte offsets (ny * Q * nx * element size just below 2^32), two z-planes
where the lattice is 3D so that the second plane's base lies above 4 GiB. Two steps of the
LES recipe (lagged Smagorinsky from the Yu strain) from a seeded random velocity field, then
populations, the emitted strain of both steps and s_nu at sampled nodes (the eight corners,
where the offsets are largest, and random nodes) against the FP64 oracle run on each node's
neighbourhood. That one more row in y is rejected for each of these boxes is checked on the
host (test_capi_host)."""
import numpy as np
import pytest

import synth
from tests._common import needs_gpu, patch_reference, pop_rel_err, sample_nodes

pytestmark = [pytest.mark.gpu, needs_gpu, pytest.mark.slow]

K = 2
LES = dict(visc="smagorinsky", drive="yu", nu0=(0.51 - 0.5) / 3.0, c_smag=0.1)

# (lattice, storage, (nz, ny, nx)): nx a multiple of 256 where possible, ny ragged
BOXES = {
    "d3q19_f32": (19, "f32", (2, 7612, 7424)),
    "d3q19_f16": (19, "f16", (1, 11037, 10240)),
    "d3q15_f32": (15, "f32", (2, 8473, 8448)),
    "d3q15_f16": (15, "f16", (2, 13981, 10240)),
    "d2q9_f32": (9, "f32", (1, 10965, 10880)),
    "d2q9_f16": (9, "f16", (1, 14563, 16384)),
}


def _spec(q, shape, storage):
    from paper_1704_07559_amd import capi
    from tests._common import spec_params
    if q == 19:
        op, cp, _ = spec_params(shape, tau=0.51, storage=storage, **LES)
        return op, cp
    if q == 15:
        from tests.test_gpu_d3q15 import _spec as spec_other
    else:
        from tests.test_gpu_d2q9 import _spec as spec_other
    op, cp = spec_other(shape, tau=0.51, **LES)
    cp.storage = {"f32": capi.LBM_F32, "f16": capi.LBM_F16, "bf16": capi.LBM_BF16}[storage]
    return op, cp


@pytest.mark.parametrize("box", sorted(BOXES))
def test_largest_box(box):
    import torch
    from oracle import d2q9, d3q15, d3q19
    from paper_1704_07559_amd import capi, lbm
    q, storage, shape = BOXES[box]
    od = {19: d3q19, 15: d3q15, 9: d2q9}[q]
    dim = 2 if q == 9 else 3
    nc = 6 if dim == 3 else 3
    op, cp = _spec(q, shape, storage)
    u = synth.random_vector(shape, seed=4242, scale=0.02)
    if dim == 2:
        u[2] = 0.0
    sim = lbm.LBM(cp, lbm.rho_u_field(np.zeros(shape), u[:dim]))
    S = [torch.empty((nc,) + shape, device="cuda") for _ in range(K)]
    for k in range(K):
        sim.step(1, S_out=S[k], strain_kind=capi.LBM_STRAIN_YU)
    nodes = sample_nodes(shape, 24, 11)
    idx = tuple(torch.tensor(a, device="cuda") for a in zip(*nodes))
    g = sim.populations()
    g_s = g[(slice(None),) + idx].double().cpu().numpy()
    del g
    S_s = [s[(slice(None),) + idx].double().cpu().numpy() for s in S]
    snu_s = sim.s_nu.reshape(shape)[idx].double().cpu().numpy()
    d = sim.reduce()
    sim.close()
    del S
    torch.cuda.empty_cache()

    def make_params(Fp):
        return od.Params(**{f: getattr(op, f) for f in op.__dataclass_fields__})

    worst_g, dS, fr, worst_s = 0.0, 0.0, 0.0, 0.0
    wts = np.array([1, 1, 1, 2, 2, 2] if dim == 3 else [1, 1, 2])
    for m, node in enumerate(nodes):
        if dim == 3:
            g_ref, S_ref, snu_ref = patch_reference(make_params, u, node, K, False, None, oracle=od)
        else:
            g_ref, S_ref, snu_ref = _patch_2d(od, make_params(None), u, node)
        worst_g = max(worst_g, pop_rel_err(g_s[:, m], g_ref, op.rho0, od.W))
        for k in range(K):
            dS = max(dS, float(np.abs(S_s[k][:, m] - S_ref[k]).max()))
            fr = max(fr, float(np.sqrt((wts * S_ref[k] ** 2).sum())))
        worst_s = max(worst_s, abs(snu_s[m] - snu_ref) / snu_ref)
    # FP16 keeps 11 significant bits of the stored deviation: a few half-ulps per step on f
    tol_g = 1e-5 if storage == "f32" else 4 * 2.0 ** -11
    tol_S = 1e-4 if storage == "f32" else 2e-2
    assert worst_g < tol_g and dS / fr < tol_S and worst_s < (1e-5 if storage == "f32" else 1e-3), \
        (worst_g, dS / fr, worst_s)
    assert d["nonfinite"] == 0


def _patch_2d(od, p, u, node):
    """D2Q9 counterpart of patch_reference: the node's (2K+1)^2 periodic neighbourhood."""
    _, _, ny, nx = u.shape
    _, y, x = node
    ix = np.ix_([0], [(y + t) % ny for t in range(-K, K + 1)], [(x + t) % nx for t in range(-K, K + 1)])
    up = np.stack([u[c][ix] for c in range(2)])
    sim = od.Simulation(p, od.init_populations(np.zeros(up.shape[1:]), up, p))
    strains = [sim.step(1)[0][:, 0, K, K].copy() for _ in range(K)]
    return sim.g[:, 0, K, K].copy(), strains, float(sim.s_nu[0, K, K])
