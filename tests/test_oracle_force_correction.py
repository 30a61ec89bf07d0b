"""Pins of the force-corrected strain (the non-equilibrium part plus half the Guo source), on
D3Q19, D2Q9 and D3Q15.

* A uniform flow under a uniform body force accelerates without deforming: its exact strain
  is zero at all times. For the LB state, write X_n = m - m^eq + S_F / 2 (S_F = T F-bar).
  Because m^eq is quadratic in j and S_F = (dm^eq/dj) . F, the forced collision followed
  by streaming maps X_n to (1 - s) X_n row by row. The corrected strain therefore decays
  geometrically: its trace at the bulk rate s_e, its deviatoric part at s_nu. The
  uncorrected strain instead settles at a value proportional to u F. The corrected one
  does not depend on the mean velocity at all. A wrong sign, a missing half, or j without
  F/2 in the source breaks both properties.
* The Yu and Chai forms stay identical (Section 5.1). The oracle corrects the moments with
  T F-bar / 2 and the distributions with F-bar / 2, on separate code paths.
* Without a force the correction changes nothing."""
import numpy as np
import pytest

import synth
from oracle import d2q9, d3q15, d3q19

LATTICES = {
    "d3q19": (d3q19, 3, 9, lambda m: d3q19.default_rates(0.8)),
    "d3q15": (d3q15, 3, 9, lambda m: d3q15.default_rates(0.8)),
    "d2q9": (d2q9, 2, 7, lambda m: d2q9.default_rates(0.8)),
}


def _trace_dev(S, dim):
    tr = S[:dim].sum(axis=0)
    dev = S.copy()
    dev[:dim] -= tr / dim
    return tr, dev


def _uniform(mod, dim, shape, u0, p):
    u = np.broadcast_to(np.asarray(u0, dtype=float).reshape((dim,) + (1,) * 3), (dim,) + shape).copy()
    return mod.Simulation(p, mod.init_populations(np.zeros(shape), u, p))


@pytest.mark.parametrize("lat", sorted(LATTICES))
def test_uniformly_accelerated_flow(lat):
    mod, dim, snu_slot, rates = LATTICES[lat]
    shape = (2, 2, 2) if dim == 3 else (1, 2, 2)
    F = np.array([2e-4, -1e-4, 3e-4])[:dim]
    u0 = np.array([0.05, -0.02, 0.03])[:dim]
    s = rates(None)
    s_e, s_nu = float(s[1]), float(s[snu_slot])
    pc = mod.Params(s=s.copy(), force=F, force_corrected=True)
    pu = mod.Params(s=s.copy(), force=F)
    sc, su = _uniform(mod, dim, shape, u0, pc), _uniform(mod, dim, shape, u0, pu)
    sc2 = _uniform(mod, dim, shape, -1.5 * u0, pc)  # another mean flow: same corrected strain
    prev = None
    for n in range(8):
        Sc = {k: sc.strain(k) for k in ("yu", "chai")}
        Su = su.strain("yu")
        # the uncorrected strain of this exactly strain-free flow is O(|u| |F|); rounding in
        # the corrected one is relative to that scale (it is a difference of such terms)
        scale = np.abs(Su).max()
        assert scale > 0.05 * np.abs(u0).max() * np.abs(F).max()
        assert np.abs(Sc["yu"] - Sc["chai"]).max() <= 1e-11 * scale
        assert np.abs(Sc["yu"] - sc2.strain("yu")).max() <= 1e-11 * scale
        tr, dev = _trace_dev(Sc["yu"], dim)
        if prev is not None:
            tr0, dev0 = prev
            assert np.abs(tr - (1 - s_e) * tr0).max() <= 1e-11 * scale, n
            assert np.abs(dev - (1 - s_nu) * dev0).max() <= 1e-11 * scale, n
            # at least 1e-4 relative resolution left at the last step
            assert min(np.abs(tr0).max(), np.abs(dev0).max()) > 1e-8 * scale
        prev = (tr, dev)
        sc.step(1)
        sc2.step(1)
        su.step(1)
    assert np.abs(prev[1]).max() > 0  # the check above is not vacuous


@pytest.mark.parametrize("lat", sorted(LATTICES))
def test_yu_equals_chai_with_a_force_field(lat):
    mod, dim, snu_slot, rates = LATTICES[lat]
    shape = (3, 4, 5) if dim == 3 else (1, 4, 5)
    Q = mod.Q
    g = synth.random_state(Q, shape, seed=31, scale=0.03)
    F = synth.uniform_random_force(shape, seed=32, amp=1e-3)[:dim]
    for visc in ("const", "smagorinsky", "smagorinsky_implicit"):
        p = mod.Params(s=rates(None), force=F, force_corrected=True, visc_kind=visc, nu0=0.01, c_smag=0.2)
        sn = np.full(shape, float(p.s[snu_slot]))
        Sy, Sc = mod.strain_of_state(g, p, sn, "yu"), mod.strain_of_state(g, p, sn, "chai")
        assert np.abs(Sy - Sc).max() <= 1e-13 * np.abs(Sy).max(), visc
        p0 = mod.Params(s=rates(None), force=F, visc_kind=visc, nu0=0.01, c_smag=0.2)
        assert np.abs(Sy - mod.strain_of_state(g, p0, sn, "yu")).max() > 1e-5 * np.abs(Sy).max()


@pytest.mark.parametrize("lat", sorted(LATTICES))
def test_no_force_no_change(lat):
    mod, dim, _, rates = LATTICES[lat]
    shape = (3, 4, 5) if dim == 3 else (1, 4, 5)
    g = synth.random_state(mod.Q, shape, seed=33, scale=0.03)
    for visc in ("const", "smagorinsky_implicit"):
        a = mod.Params(s=rates(None), force_corrected=True, visc_kind=visc, nu0=0.01, c_smag=0.2)
        b = mod.Params(s=rates(None), visc_kind=visc, nu0=0.01, c_smag=0.2)
        sa = mod.Simulation(a, g.copy())
        sb = mod.Simulation(b, g.copy())
        for _ in range(3):
            assert np.array_equal(sa.strain("yu"), sb.strain("yu"))
            assert np.array_equal(sa.strain("chai"), sb.strain("chai"))
            sa.step(1)
            sb.step(1)
        assert np.array_equal(sa.g, sb.g)


def test_implicit_coupling_with_correction_is_a_fixed_point():
    shape = (3, 4, 5)
    g = synth.random_state(19, shape, seed=34, scale=0.02)
    F = synth.uniform_random_force(shape, seed=35, amp=1e-3)
    for drive in ("yu", "chai"):
        p = d3q19.Params(visc_kind="smagorinsky_implicit", visc_strain=drive, nu0=0.002, c_smag=0.3, force=F,
                         force_corrected=True)
        out = d3q19.collide(g, p, np.full(shape, p.s[9]))
        S = out.S_yu if drive == "yu" else out.S_chai
        lhs = out.s_nu * (3.0 * (p.nu0 + p.c_smag**2 * np.sqrt(2.0 * d3q19.strain_sq(S))) + 0.5)
        assert np.abs(lhs - 1.0).max() < 1e-14
