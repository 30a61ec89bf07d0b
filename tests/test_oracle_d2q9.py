"""Pins of the D2Q9 oracle (Sections 5.3 and 5.4: the Chai formula on another lattice and
the Yu-type formula derived from it)."""
import numpy as np
import pytest
import sympy as sp

import synth
from oracle import closed_forms as cf
from oracle import d2q9 as d


def test_transform_orthogonal_and_inverse():
    G = d.T @ d.T.T
    assert np.abs(G - np.diag(np.diag(G))).max() == 0
    assert np.array_equal(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])
    assert np.abs(d.T @ d.TINV - np.eye(9)).max() <= 9 * np.finfo(float).eps


def test_weights_and_equilibrium_identities():
    """sum w = 1, sum w c c = c_s^2 I; Eq. cfeqmoment_ holds on D2Q9 (Section 5.3 relies
    on it): sum c c g^eq = c_s^2 drho I + rho0 u u, and the third moment."""
    Cf = d.C.astype(float)
    assert abs(d.W.sum() - 1) < 1e-15
    assert np.abs((Cf * d.W) @ Cf.T - d.CS2 * np.eye(2)).max() < 1e-15
    rng = np.random.default_rng(1)
    dr, r0 = 0.013, 1.4
    u = rng.normal(size=2) * 0.05
    ge = d.g_eq(np.array(dr), r0 * u, r0)
    P2 = np.einsum("ai,bi,i->ab", Cf, Cf, ge)
    assert np.abs(P2 - (d.CS2 * dr * np.eye(2) + r0 * np.outer(u, u))).max() < 1e-16
    P3 = np.einsum("ai,bi,ci,i->abc", Cf, Cf, Cf, ge)
    I = np.eye(2)
    ref = d.CS2 * r0 * (np.einsum("ab,c->abc", I, u) + np.einsum("ac,b->abc", I, u) + np.einsum("bc,a->abc", I, u))
    assert np.abs(P3 - ref).max() < 1e-16


def test_m_eq_is_T_of_g_eq():
    rng = np.random.default_rng(2)
    dr = rng.normal(size=(3, 4)) * 0.02
    j = rng.normal(size=(2, 3, 4)) * 0.05
    for r0 in (1.0, 1.9):
        assert np.abs(np.tensordot(d.T, d.g_eq(dr, j, r0), axes=(1, 0)) - d.m_eq(dr, j, r0)).max() < 1e-16


def test_section_5_4_route_gives_the_closed_form_yu_type_formula():
    """Carrying out Section 5.4 symbolically (exact rationals) on D2Q9 gives
    S_xx = -(s_e m1 + 3 s_nu m7) / (4 rho0), S_yy = -(s_e m1 - 3 s_nu m7) / (4 rho0),
    S_xy = -3 s_nu m8 / (2 rho0); the oracle's numerical route agrees."""
    Ts = sp.Matrix(d.T.astype(int).tolist())
    m = sp.symbols("m0:9")
    s_c, s_e, s_eps, s_q, s_nu, rho0 = sp.symbols("s_c s_e s_eps s_q s_nu rho0", positive=True)
    L = sp.diag(s_c, s_e, s_eps, s_c, s_q, s_c, s_q, s_nu, s_nu)
    m1 = sp.Matrix([0, m[1], m[2], 0, m[4], 0, m[6], m[7], m[8]])  # conserved rows have no neq part
    M = Ts.inv() * L * m1
    cs2 = sp.Rational(1, 3)
    S = {}
    for name, (a, b) in (("xx", (0, 0)), ("yy", (1, 1)), ("xy", (0, 1))):
        N = sum(int(d.C[a, i]) * int(d.C[b, i]) * M[i] for i in range(9))
        S[name] = sp.simplify(-N / (2 * rho0 * cs2))
    assert sp.simplify(S["xx"] + (s_e * m[1] + 3 * s_nu * m[7]) / (4 * rho0)) == 0
    assert sp.simplify(S["yy"] + (s_e * m[1] - 3 * s_nu * m[7]) / (4 * rho0)) == 0
    assert sp.simplify(S["xy"] + 3 * s_nu * m[8] / (2 * rho0)) == 0
    rng = np.random.default_rng(3)
    mv = rng.normal(size=9)
    mv[[0, 3, 5]] = 0
    s = d.default_rates(0.7)
    r = 1.3
    num = d.strain_yu_type(mv, s, r)
    ref = [-(s[1] * mv[1] + 3 * s[7] * mv[7]) / (4 * r), -(s[1] * mv[1] - 3 * s[7] * mv[7]) / (4 * r),
           -3 * s[7] * mv[8] / (2 * r)]
    assert np.abs(num - np.array(ref)).max() < 4 * np.finfo(float).eps * np.abs(ref).max()


def test_yu_type_equals_chai_on_arbitrary_states():
    rng = np.random.default_rng(4)
    shape = (1, 5, 6)
    for t in range(3):
        s = d.default_rates(1.0 / (0.6 + rng.random()))
        s[[1, 2, 4, 6]] = 0.5 + rng.random(4) * 1.4
        p = d.Params(rho0=0.8 + rng.random(), s=s)
        g = synth.random_state(9, shape, seed=t, scale=0.05)
        sn = np.full(shape, s[7])
        Sy, Sc = d.strain_of_state(g, p, sn, "yu"), d.strain_of_state(g, p, sn, "chai")
        assert np.abs(Sy - Sc).max() <= 1e-14 * np.abs(Sy).max()


def test_srt_limit():
    tau = 0.77
    p = d.Params(s=np.full(9, 1 / tau))
    shape = (1, 3, 4)
    g = synth.random_state(9, shape, seed=5, scale=0.03)
    g_post, Sy, Sc, _ = d.collide(g, p, np.full(shape, 1 / tau))
    drho, j = d.macroscopic(g)
    ge = d.g_eq(drho, j, p.rho0)
    assert np.abs(g_post - (g - (g - ge) / tau)).max() < 1e-15
    Cf = d.C.astype(float)
    ref = np.stack([-np.tensordot(Cf[a] * Cf[b], g - ge, axes=(0, 0)) / (2 * d.CS2 * tau) for a, b in ((0, 0), (1, 1), (0, 1))])
    assert np.abs(Sc - ref).max() < 1e-15


def test_conservation_with_force_and_walls():
    shape = (1, 8, 7)
    F = synth.random_vector(shape, seed=6, scale=1e-4)[:2]
    p = d.Params(force=F, visc_kind="smagorinsky", nu0=0.01)
    u = synth.random_vector(shape, seed=7, scale=0.02)[:2]
    sim = d.Simulation(p, d.init_populations(np.zeros(shape), u, p))
    m0 = sim.g.sum()
    mom0 = np.tensordot(d.C.astype(float), sim.g, axes=(1, 0)).reshape(2, -1).sum(1)
    sim.step(20)
    assert abs(sim.g.sum() - m0) < 1e-14
    mom1 = np.tensordot(d.C.astype(float), sim.g, axes=(1, 0)).reshape(2, -1).sum(1)
    assert np.abs(mom1 - mom0 - 20 * F.reshape(2, -1).sum(1)).max() < 1e-15
    pw = d.Params(walls_y=True, force=np.array([1e-4, 0.0]))
    sw = d.Simulation(pw, d.init_populations(np.zeros(shape), u, pw))
    m0 = sw.g.sum()
    sw.step(20)
    assert abs(sw.g.sum() - m0) < 1e-14


def test_second_order_convergence_of_S_xy_d2q9():
    """Rotated Taylor-Green vortex on D2Q9 under diffusive scaling, N = 16, 32, 64."""
    tau = 0.8
    errs = []
    for N in (16, 32, 64):
        u0 = 0.05 * 32 / N
        steps = int(round(200 * (N / 32) ** 2))
        shape = (1, N, N)
        dr, u, gu = synth.tgv_rotated(shape, u0, 1.0)
        p = d.Params(s=d.default_rates(tau))
        sim = d.Simulation(p, d.init_populations(dr, u[:2], p, gu[:2, :2]))
        exact0 = cf.tgv_rotated_strain(shape, u0, cf.nu_of_rate(1 / tau), 0)[3]
        assert np.abs(sim.strain("chai")[2] - exact0).max() < 1e-14
        sim.step(steps)
        exact = cf.tgv_rotated_strain(shape, u0, cf.nu_of_rate(1 / tau), steps)[3]
        errs.append(np.linalg.norm(sim.strain("yu")[2] - exact) / np.linalg.norm(exact))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (orders >= 1.8).all(), (errs, orders)


def test_implicit_smagorinsky_rate_is_a_fixed_point():
    """The non-lagged coupling: the solved s_nu satisfies s = 1/(3 (nu0 + C^2 |S(s)|) + 1/2)
    to FP64 resolution for either driving formula, both formulas agree at the solved rate,
    and C_s = 0 recovers the molecular rate."""
    shape = (1, 5, 7)
    g = synth.random_state(9, shape, seed=41, scale=0.02)
    for drive in ("yu", "chai"):
        p = d.Params(visc_kind="smagorinsky_implicit", visc_strain=drive, nu0=0.002, c_smag=0.3)
        _, S_yu, S_chai, s_nu = d.collide(g, p, np.full(shape, p.s[7]))
        S = S_yu if drive == "yu" else S_chai
        lhs = s_nu * (3.0 * (p.nu0 + p.c_smag**2 * np.sqrt(2.0 * d.strain_sq(S))) + 0.5)
        assert np.abs(lhs - 1.0).max() < 1e-14
        assert np.abs(S_yu - S_chai).max() <= 1e-13 * np.abs(S_yu).max()
        assert np.abs(d.strain_of_state(g, p, np.full(shape, p.s[7]), drive) - S).max() == 0.0
        p0 = d.Params(visc_kind="smagorinsky_implicit", visc_strain=drive, nu0=0.1, c_smag=0.0)
        assert np.abs(d.collide(g, p0, np.full(shape, p.s[7]))[3] - 1.0 / 0.8).max() < 1e-14


def test_implicit_smagorinsky_conserves():
    shape = (1, 5, 7)
    p = d.Params(visc_kind="smagorinsky_implicit", nu0=0.01, c_smag=0.2)
    u = synth.random_vector(shape, seed=42, scale=0.03)[:2]
    sim = d.Simulation(p, d.init_populations(np.zeros(shape), u, p))
    m0 = sim.g.sum()
    j0 = np.tensordot(d.C.astype(float), sim.g, axes=(1, 0)).reshape(2, -1).sum(1)
    sim.step(20)
    assert abs(sim.g.sum() - m0) < 1e-13
    j1 = np.tensordot(d.C.astype(float), sim.g, axes=(1, 0)).reshape(2, -1).sum(1)
    assert np.abs(j1 - j0).max() < 1e-13


def test_naive_loop_matches_vectorised_step():
    """Brute force: the per-node loop (explicit neighbour indices, the closed-form Yu-type
    formula, an explicit per-node T^-1 diag(s) T) reproduces the vectorised D2Q9 step, with
    walls, a force field and variable viscosity."""
    from oracle import naive_other
    shape = (1, 5, 6)
    for kw in (dict(), dict(visc_kind="smagorinsky", nu0=0.02, c_smag=0.3),
               dict(visc_kind="powerlaw", visc_strain="chai", K_pl=0.02, n_pl=1.4, walls_y=True,
                    force=synth.random_vector(shape, seed=5, scale=1e-3)[:2])):
        p = d.Params(**kw)
        g = synth.random_state(9, shape, seed=7, scale=0.01)
        sn = np.full(shape, p.s[7]) * (1 + 0.1 * synth.random_vector(shape, seed=9, scale=1.0)[0])
        g_post, S_yu, S_chai, s_nu = d.collide(g, p, sn)
        nxt = d.stream(g_post, p.walls_y)
        g2, Sy, Sc, snew = naive_other.step(d, g, p, sn)
        assert np.abs(nxt - g2).max() < 1e-15
        assert np.abs(S_yu - Sy).max() < 1e-15
        assert np.abs(S_chai - Sc).max() < 1e-15
        assert np.abs(s_nu - snew).max() < 1e-14


def test_chapman_enskog_prediction_of_the_nonequilibrium_moments():
    """The non-equilibrium moments the Section 5.4 Yu-type formula inverts (ce_neq_moments)
    are what the D2Q9 dynamics produce on a smooth flow: started from the plain equilibrium,
    the measured m - m^eq approaches the prediction from grad u at about second order."""
    tau, e = 0.8, []
    for N in (16, 32, 64):
        shape = (1, N, N)
        u0 = 0.02 * 16 / N
        steps = int(60 * (N / 16) ** 2)
        dr, u, gu = synth.tgv_rotated(shape, u0, 1.0)
        p = d.Params(s=d.default_rates(tau))
        sim = d.Simulation(p, d.init_populations(dr, u[:2], p))
        sim.step(steps)
        k = 2.0 * np.pi / N
        dec = np.exp(-cf.nu_of_rate(1 / tau) * k * k * steps)
        drho, j = d.macroscopic(sim.g)
        mneq = np.tensordot(d.T, sim.g, axes=(1, 0)) - d.m_eq(drho, j, p.rho0)
        pred = d.ce_neq_moments(gu[:2, :2] * dec, p, float(p.s[7]))
        rows = [1, 7, 8]
        e.append(np.abs(mneq[rows] - pred[rows]).max() / np.abs(pred[rows]).max())
    assert e[-1] < 5e-3, e
    assert all(np.log2(a / b) > 1.7 for a, b in zip(e[:-1], e[1:])), e
