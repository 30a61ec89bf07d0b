"""Pins of the FP64 adjoint oracle for strain-dependent viscosities (lagged Smagorinsky,
lagged power law, implicit Smagorinsky): every derivative against central differences of
the pinned forward oracle, the whole gradient against finite differences of the loss, and
the constant-viscosity adjoint as the limit C_s = 0."""
import numpy as np
import pytest

import synth
from oracle import adjoint as adj
from oracle import adjoint_visc as av
from oracle import d3q19 as d


def _fd(f, h):
    """Fourth-order central difference at 0."""
    return (8.0 * (f(h) - f(-h)) - (f(2 * h) - f(-2 * h))) / (12.0 * h)


MODELS = {
    "smag_yu": dict(visc_kind="smagorinsky", visc_strain="yu", nu0=0.01, c_smag=0.4),
    "smag_chai": dict(visc_kind="smagorinsky", visc_strain="chai", nu0=0.002, c_smag=0.3),
    "powerlaw_thinning": dict(visc_kind="powerlaw", visc_strain="chai", K_pl=0.02, n_pl=0.5, nu_min=1e-3, nu_max=0.5),
    "powerlaw_thickening": dict(visc_kind="powerlaw", visc_strain="yu", K_pl=2.0, n_pl=1.5, nu_min=1e-3, nu_max=1.0),
    "implicit_yu": dict(visc_kind="smagorinsky_implicit", visc_strain="yu", nu0=0.01, c_smag=0.4),
    "implicit_chai": dict(visc_kind="smagorinsky_implicit", visc_strain="chai", nu0=0.002, c_smag=0.3),
}


def _params(name, walls=False):
    p = d.Params(s=d.default_rates(0.8), walls_y=walls, **MODELS[name])
    return p


def _state(shape, seed, p):
    u = synth.random_vector(shape, seed=seed, scale=0.05)
    return d.init_populations(np.zeros(shape), u, p) + synth.random_state(19, shape, seed=seed + 1, scale=3e-3)


def _lagged(p):
    return p.visc_kind != "smagorinsky_implicit"


def _s_prev(shape, seed, p):
    return 1.0 / (3.0 * (0.02 + 0.01 * synth.random_state(1, shape, seed=seed, scale=1.0)[0] ** 2) + 0.5)


@pytest.mark.parametrize("name", sorted(MODELS))
def test_collision_derivatives_against_central_differences(name):
    """dg*/dg, dg*/dF, dg*/ds_prev and ds_new/d(g, F, s_prev) of collision_jacobians_visc
    against fourth-order central differences of d3q19.collide."""
    shape = (2, 3, 4)
    p = _params(name)
    g = _state(shape, 3, p)
    F = synth.random_vector(shape, seed=4, scale=1e-4)
    sp = _s_prev(shape, 5, p)
    Jv = av.collision_jacobians_visc(g, sp if _lagged(p) else None, F, p)

    def run(dg=0.0, dF=0.0, ds=0.0):
        out = d.collide(g + dg, adj._with_force(p, F + dF), sp + ds)
        return out.g_post, out.s_nu

    assert np.abs(run()[1].reshape(-1) - Jv["s"]).max() < 1e-14
    v = synth.random_state(19, shape, seed=6, scale=1.0)
    vF = synth.random_vector(shape, seed=7, scale=1.0)
    vs = synth.random_state(1, shape, seed=8, scale=1.0)[0]
    h = 1e-6
    cases = [
        (lambda t: run(dg=t * v), np.einsum("mil,lm->im", Jv["Jgg"], v.reshape(19, -1)),
         (Jv["ds_dg"] * v.reshape(19, -1).T).sum(axis=1), h),
        (lambda t: run(dF=t * vF), np.einsum("mik,km->im", Jv["JgF"], vF.reshape(3, -1)),
         (Jv["ds_dF"] * vF.reshape(3, -1).T).sum(axis=1), 1e-5),
    ]
    if _lagged(p):
        cases.append((lambda t: run(ds=t * vs), Jv["Jgs"] * vs.reshape(-1), Jv["ds_dsp"] * vs.reshape(-1), 1e-6))
    for f, dg_ref, ds_ref, hh in cases:
        dg_fd = _fd(lambda t: f(t)[0], hh).reshape(19, -1)
        ds_fd = _fd(lambda t: f(t)[1], hh).reshape(-1)
        assert np.abs(dg_fd - dg_ref).max() <= 1e-8 * np.abs(dg_ref).max()
        assert np.abs(ds_fd - ds_ref).max() <= 1e-8 * np.abs(ds_ref).max() + 1e-15
    # the rate really moves with the state (the test is not vacuous)
    assert np.abs(Jv["ds_dg"]).max() > 1e-3


def test_power_law_clamps_have_zero_slope():
    shape = (2, 2, 3)
    p = d.Params(s=d.default_rates(0.8), visc_kind="powerlaw", visc_strain="yu", K_pl=0.02, n_pl=0.5,
                 nu_min=1e-3, nu_max=0.02)
    g = _state(shape, 9, p)
    F = np.zeros((3,) + shape)
    Jv = av.collision_jacobians_visc(g, _s_prev(shape, 10, p), F, p)
    assert np.allclose(Jv["s"], 1.0 / (3.0 * 0.02 + 0.5))   # every node at nu_max
    assert np.abs(Jv["ds_dg"]).max() == 0.0 and np.abs(Jv["ds_dsp"]).max() == 0.0


@pytest.mark.parametrize("name", ["smag_yu", "powerlaw_thinning", "implicit_chai"])
@pytest.mark.parametrize("walls", [False, True])
def test_adjoint_step_dot_product(name, walls):
    """<L v, w> = <v, L^T w> for the linearised step (g, s_prev, F) -> (g^{n+1}, s_new),
    L v from central differences of the forward oracle."""
    shape = (3, 4, 5)
    p = _params(name, walls)
    g = _state(shape, 11, p)
    F = synth.random_vector(shape, seed=12, scale=1e-4)
    sp = _s_prev(shape, 13, p)
    lag = _lagged(p)

    def step(t, v, vF, vs):
        out = d.collide(g + t * v, adj._with_force(p, F + t * vF), sp + t * vs)
        return d.stream(out.g_post, walls), out.s_nu

    v = synth.random_state(19, shape, seed=14, scale=1.0)
    vF = synth.random_vector(shape, seed=15, scale=1.0)
    vs = synth.random_state(1, shape, seed=16, scale=1.0)[0]
    w = synth.random_state(19, shape, seed=17, scale=1.0)
    ws = synth.random_state(1, shape, seed=18, scale=1.0)[0]
    lam, lams, gF = av.adjoint_step_visc(w, ws if lag else None, g, sp if lag else None, F, p)
    z, zF, zs = np.zeros_like(v), np.zeros_like(vF), np.zeros_like(vs)
    dirs = [((v, zF, zs), (v * lam).sum(), 1e-6), ((z, vF, zs), (vF * gF).sum(), 1e-5)]
    if lag:
        dirs.append(((z, zF, vs), (vs * lams).sum(), 1e-6))
    for (a, aF, as_), rhs, h in dirs:
        Lg = _fd(lambda t: step(t, a, aF, as_)[0], h)
        Ls = _fd(lambda t: step(t, a, aF, as_)[1], h)
        lhs = (Lg * w).sum() + ((Ls * ws).sum() if lag else 0.0)
        assert abs(lhs - rhs) <= 1e-8 * abs(lhs)


@pytest.mark.parametrize("name", ["smag_chai", "powerlaw_thickening", "implicit_yu"])
def test_loss_seed_against_finite_differences(name):
    shape = (3, 4, 5)
    p = _params(name)
    g = _state(shape, 19, p)
    F = synth.random_vector(shape, seed=20, scale=1e-3)
    sp = _s_prev(shape, 21, p)
    lag = _lagged(p)

    def loss(dg=0.0, dF=0.0, ds=0.0):
        return float(d.strain_sq(d.strain_of_state(g + dg, adj._with_force(p, F + dF), sp + ds, "yu")).sum())

    J, lam, lams, gF = av.strain_loss_seed_visc(g, sp if lag else None, F, p)
    assert abs(J - loss()) <= 1e-13 * J
    v = synth.random_state(19, shape, seed=22, scale=1.0)
    vF = synth.random_vector(shape, seed=23, scale=1.0)
    assert abs(_fd(lambda t: loss(dg=t * v), 1e-6) - (lam * v).sum()) <= 1e-8 * abs((lam * v).sum())
    assert abs(_fd(lambda t: loss(dF=t * vF), 1e-5) - (gF * vF).sum()) <= 1e-8 * abs((gF * vF).sum())
    if lag:
        vs = synth.random_state(1, shape, seed=24, scale=1.0)[0]
        assert abs(_fd(lambda t: loss(ds=t * vs), 1e-6) - (lams * vs).sum()) <= 1e-8 * abs((lams * vs).sum())


def _problem(n=6, seed_u=1704, seed_f=7559):
    shape = (n, n + 1, n + 2)
    u0 = 0.05 * synth.random_vector(shape, seed=seed_u, scale=1.0)
    F = synth.uniform_random_force(shape, seed=seed_f, amp=1e-5)
    return u0, F


@pytest.mark.parametrize("name,walls", [("smag_yu", False), ("powerlaw_thinning", True), ("implicit_chai", False)])
def test_gradient_against_finite_differences(name, walls):
    """Whole-run gradient (12 steps, checkpoint every 5) against fourth-order central
    differences of the forward loss, directional in u0 and F and at single entries."""
    p = _params(name, walls)
    u0, F = _problem()
    nsteps = 12
    J, gu, gF = adj.gradient(u0, F, p, nsteps, every=5)
    assert abs(J - adj.forward(u0, F, p, nsteps)) <= 1e-12 * J
    du = synth.random_vector(u0.shape[1:], seed=3, scale=1.0)
    fd = _fd(lambda t: adj.forward(u0 + t * du, F, p, nsteps), 1e-6)
    assert abs(fd - (gu * du).sum()) <= 1e-7 * abs(fd)
    dF = synth.random_vector(u0.shape[1:], seed=4, scale=1.0)
    # |S| is not smooth where S vanishes: steps well below the smallest local strain
    fdF = _fd(lambda t: adj.forward(u0, F + t * dF, p, nsteps), 1e-7)
    assert abs(fdF - (gF * dF).sum()) <= 1e-7 * abs(fdF)
    e = np.zeros_like(u0)
    e[1, 2, 3, 4] = 1.0
    fdp = _fd(lambda t: adj.forward(u0 + t * e, F, p, nsteps), 1e-6)
    assert abs(fdp - gu[1, 2, 3, 4]) <= 1e-7 * np.abs(gu).max()


def test_zero_smagorinsky_constant_reduces_to_the_constant_viscosity_adjoint():
    """C_s = 0: the lagged and implicit models are the constant viscosity nu0, so their
    gradients equal the constant-viscosity adjoint with s_nu = 1/(3 nu0 + 1/2)."""
    u0, F = _problem(n=4)
    nu0 = 0.05
    s_nu = 1.0 / (3.0 * nu0 + 0.5)
    pc = d.Params(s=d.default_rates(1.0 / s_nu))
    ref = adj.gradient(u0, F, pc, 6, every=4)
    for kind in ("smagorinsky", "smagorinsky_implicit"):
        p = d.Params(s=d.default_rates(1.0 / s_nu), visc_kind=kind, nu0=nu0, c_smag=0.0)
        got = adj.gradient(u0, F, p, 6, every=4)
        assert abs(got[0] - ref[0]) <= 1e-13 * ref[0]
        assert np.abs(got[1] - ref[1]).max() <= 1e-11 * np.abs(ref[1]).max()
        assert np.abs(got[2] - ref[2]).max() <= 1e-11 * np.abs(ref[2]).max()


def test_checkpointing_recomputes_bit_identically():
    u0, F = _problem(n=4)
    p = _params("smag_yu")
    a = adj.gradient(u0, F, p, 9, every=None)
    b = adj.gradient(u0, F, p, 9, every=4)
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
