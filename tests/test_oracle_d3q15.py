"""Pins of the D3Q15 oracle (Sections 5.3 and 5.4: the Chai formula on another lattice and
the Yu-type formula derived from it by the Section 5.4 route)."""
import numpy as np
import pytest
import sympy as sp

import synth
from oracle import closed_forms as cf
from oracle import d3q15 as d


def test_transform_is_the_dhumieres_basis():
    """Rows orthogonal with norms (15, 18, 360, 10, 40, 10, 40, 10, 40, 12, 4, 8, 8, 8, 8);
    the published integer rows of e, eps and q_x (rest / faces / corners); T T^-1 = I."""
    G = d.T @ d.T.T
    assert np.abs(G - np.diag(np.diag(G))).max() == 0
    assert np.array_equal(np.diag(G), [15, 18, 360, 10, 40, 10, 40, 10, 40, 12, 4, 8, 8, 8, 8])
    faces, corners = slice(1, 7), slice(7, 15)
    assert d.T[1, 0] == -2 and (d.T[1, faces] == -1).all() and (d.T[1, corners] == 1).all()
    assert d.T[2, 0] == 16 and (d.T[2, faces] == -4).all() and (d.T[2, corners] == 1).all()
    assert np.array_equal(d.T[4, faces], -4 * d.C[0, faces]) and np.array_equal(d.T[4, corners], d.C[0, corners])
    assert np.abs(d.T @ d.TINV - np.eye(15)).max() <= 15 * np.finfo(float).eps
    assert all(d.OPP[d.OPP[i]] == i and (d.C[:, d.OPP[i]] == -d.C[:, i]).all() for i in range(15))


def test_weights_and_equilibrium_identities():
    """Lattice isotropy to fourth order, and Eq. cfeqmoment_ (which Section 5.3 relies on):
    sum c c g^eq = c_s^2 drho I + rho0 u u, sum c c c g^eq = c_s^2 rho0 (u d + d u + ...)."""
    Cf = d.C.astype(float)
    assert abs(d.W.sum() - 1) < 1e-15
    assert np.abs((Cf * d.W) @ Cf.T - d.CS2 * np.eye(3)).max() < 1e-15
    c4 = np.einsum("i,ai,bi,ci,di->abcd", d.W, Cf, Cf, Cf, Cf)
    I = np.eye(3)
    ref4 = d.CS2**2 * (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I) + np.einsum("ad,bc->abcd", I, I))
    assert np.abs(c4 - ref4).max() < 1e-15
    rng = np.random.default_rng(1)
    dr, r0 = 0.013, 1.4
    u = rng.normal(size=3) * 0.05
    ge = d.g_eq(np.array(dr), r0 * u, r0)
    P2 = np.einsum("ai,bi,i->ab", Cf, Cf, ge)
    assert np.abs(P2 - (d.CS2 * dr * I + r0 * np.outer(u, u))).max() < 1e-16
    P3 = np.einsum("ai,bi,ci,i->abc", Cf, Cf, Cf, ge)
    ref = d.CS2 * r0 * (np.einsum("ab,c->abc", I, u) + np.einsum("ac,b->abc", I, u) + np.einsum("bc,a->abc", I, u))
    assert np.abs(P3 - ref).max() < 1e-16


def test_m_eq_is_T_of_g_eq_and_guo_moments():
    rng = np.random.default_rng(2)
    dr = rng.normal(size=(3, 4)) * 0.02
    j = rng.normal(size=(3, 3, 4)) * 0.05
    F = rng.normal(size=(3, 3, 4)) * 1e-3
    for r0 in (1.0, 1.9):
        assert np.abs(d.moments(d.g_eq(dr, j, r0)) - d.m_eq(dr, j, r0)).max() < 1e-16
        # T F-bar = (d m^eq / d j) . F (m^eq quadratic in j: the central difference is exact)
        lin = (d.m_eq(dr, j + F, r0) - d.m_eq(dr, j - F, r0)) / 2.0
        assert np.abs(d.moments(d.guo_force_populations(j, F, r0)) - lin).max() < 1e-13 * np.abs(lin).max()


def test_section_5_4_route_gives_the_closed_form_yu_type_formula():
    """Carrying out Section 5.4 symbolically (exact rationals) on D3Q15 gives
      S_xx = -(s_e m1 + s_nu m9) / (2 rho0),
      S_yy = -(2 s_e m1 - s_nu m9 + 3 s_nu m10) / (4 rho0),
      S_zz = -(2 s_e m1 - s_nu m9 - 3 s_nu m10) / (4 rho0),
      S_xy, S_yz, S_xz = -3 s_nu m11, m12, m13 / (2 rho0),
    independent of s_eps, s_q and s_m; the oracle's numerical route agrees."""
    Ts = sp.Matrix(d.T.astype(int).tolist())
    m = sp.symbols("m0:15")
    s_e, s_eps, s_q, s_nu, s_m, rho0 = sp.symbols("s_e s_eps s_q s_nu s_m rho0", positive=True)
    L = sp.diag(0, s_e, s_eps, 0, s_q, 0, s_q, 0, s_q, s_nu, s_nu, s_nu, s_nu, s_nu, s_m)
    m1 = sp.Matrix([0, m[1], m[2], 0, m[4], 0, m[6], 0, m[8]] + list(m[9:15]))
    M = Ts.inv() * L * m1
    cs2 = sp.Rational(1, 3)
    expect = {
        (0, 0): -(s_e * m[1] + s_nu * m[9]) / (2 * rho0),
        (1, 1): -(2 * s_e * m[1] - s_nu * m[9] + 3 * s_nu * m[10]) / (4 * rho0),
        (2, 2): -(2 * s_e * m[1] - s_nu * m[9] - 3 * s_nu * m[10]) / (4 * rho0),
        (0, 1): -3 * s_nu * m[11] / (2 * rho0),
        (1, 2): -3 * s_nu * m[12] / (2 * rho0),
        (0, 2): -3 * s_nu * m[13] / (2 * rho0),
    }
    for (a, b), ref in expect.items():
        N = sum(int(d.C[a, i]) * int(d.C[b, i]) * M[i] for i in range(15))
        assert sp.simplify(-N / (2 * rho0 * cs2) - ref) == 0
    rng = np.random.default_rng(3)
    mv = rng.normal(size=15)
    mv[[0, 3, 5, 7]] = 0
    s = d.default_rates(0.7)
    r = 1.3
    num = d.strain_yu_type(mv, s, r)
    ref = np.array([float(e.subs({rho0: r, s_e: s[1], s_nu: s[9], **{m[k]: mv[k] for k in range(15)}}))
                    for e in expect.values()])
    assert np.abs(num - ref).max() < 8 * np.finfo(float).eps * np.abs(ref).max()


def test_yu_type_equals_chai_on_arbitrary_states():
    """Section 5.1's identity carries over: both formulas agree for any state, force, rates."""
    rng = np.random.default_rng(4)
    shape = (3, 5, 6)
    for t in range(3):
        s = d.default_rates(1.0 / (0.6 + rng.random()))
        s[[1, 2, 4, 6, 8, 14]] = 0.5 + rng.random(6) * 1.4
        p = d.Params(rho0=0.8 + rng.random(), s=s, force=synth.random_vector(shape, seed=10 + t, scale=1e-3))
        g = synth.random_state(15, shape, seed=t, scale=0.05)
        sn = np.full(shape, s[9])
        Sy, Sc = d.strain_of_state(g, p, sn, "yu"), d.strain_of_state(g, p, sn, "chai")
        assert np.abs(Sy - Sc).max() <= 1e-14 * np.abs(Sy).max()


def test_srt_limit():
    """All rates 1/tau: the collision is BGK and the Chai strain is Eq. ChaiS_srt."""
    tau = 0.77
    p = d.Params(s=np.full(15, 1 / tau))
    shape = (2, 3, 4)
    g = synth.random_state(15, shape, seed=5, scale=0.03)
    g_post, Sy, Sc, _ = d.collide(g, p, np.full(shape, 1 / tau))
    drho, j = d.macroscopic(g)
    ge = d.g_eq(drho, j, p.rho0)
    assert np.abs(g_post - (g - (g - ge) / tau)).max() < 1e-15
    Cf = d.C.astype(float)
    ref = np.stack([-np.tensordot(Cf[a] * Cf[b], g - ge, axes=(0, 0)) / (2 * d.CS2 * tau)
                    for a, b in ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2))])
    assert np.abs(Sc - ref).max() < 1e-15


def test_conservation_with_force_and_walls():
    shape = (4, 8, 7)
    F = synth.random_vector(shape, seed=6, scale=1e-4)
    p = d.Params(force=F, visc_kind="smagorinsky", nu0=0.01)
    u = synth.random_vector(shape, seed=7, scale=0.02)
    sim = d.Simulation(p, d.init_populations(np.zeros(shape), u, p))
    m0 = sim.g.sum()
    mom0 = np.tensordot(d.C.astype(float), sim.g, axes=(1, 0)).reshape(3, -1).sum(1)
    sim.step(20)
    assert abs(sim.g.sum() - m0) < 1e-13
    mom1 = np.tensordot(d.C.astype(float), sim.g, axes=(1, 0)).reshape(3, -1).sum(1)
    assert np.abs(mom1 - mom0 - 20 * F.reshape(3, -1).sum(1)).max() < 1e-14
    pw = d.Params(walls_y=True, force=np.array([0.0, 0.0, 1e-4]), visc_kind="powerlaw", visc_strain="chai",
                  K_pl=0.02, n_pl=0.6)
    sw = d.Simulation(pw, d.init_populations(np.zeros(shape), u, pw))
    m0 = sw.g.sum()
    sw.step(20)
    assert abs(sw.g.sum() - m0) < 1e-13


def _tgv_error(N, plane, kind, tau=0.8):
    u0 = 0.05 * 32 / N
    steps = int(round(200 * (N / 32) ** 2))
    shape = [1, 1, 1]
    for a in plane:
        shape[2 - a] = N
    shape = tuple(shape)
    p = d.Params(s=d.default_rates(tau))
    dr, u, gu = synth.tgv_rotated(shape, u0, 1.0, plane)
    sim = d.Simulation(p, d.init_populations(dr, u, p, gu))
    exact0 = cf.tgv_rotated_strain(shape, u0, cf.nu_of_rate(1 / tau), 0.0, plane)
    assert np.abs(sim.strain(kind) - exact0).max() < 1e-14  # the CE initial state gives S exactly
    sim.step(steps)
    exact = cf.tgv_rotated_strain(shape, u0, cf.nu_of_rate(1 / tau), steps, plane)
    comp = {(0, 1): 3, (1, 2): 4, (0, 2): 5}[plane]
    S = sim.strain(kind)
    return np.linalg.norm(S[comp] - exact[comp]) / np.linalg.norm(exact[comp])


@pytest.mark.slow
@pytest.mark.parametrize("plane,kind", [((0, 1), "yu"), ((1, 2), "chai"), ((0, 2), "yu")])
def test_second_order_convergence_of_the_off_diagonal_strain(plane, kind):
    """Rotated Taylor-Green vortex in each coordinate plane, diffusive scaling N = 16, 32, 64:
    the D3Q15 strain converges at second order like the D3Q19 one (Section 5.1)."""
    e = [_tgv_error(N, plane, kind) for N in (16, 32, 64)]
    orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert (orders >= 1.8).all(), (e, orders)


def test_implicit_smagorinsky_rate_is_a_fixed_point():
    """The non-lagged coupling: the solved s_nu satisfies s = 1/(3 (nu0 + C^2 |S(s)|) + 1/2)
    to FP64 resolution for either driving formula, both formulas agree at the solved rate,
    and C_s = 0 recovers the molecular rate."""
    shape = (3, 5, 7)
    g = synth.random_state(15, shape, seed=41, scale=0.02)
    for drive in ("yu", "chai"):
        p = d.Params(visc_kind="smagorinsky_implicit", visc_strain=drive, nu0=0.002, c_smag=0.3)
        _, S_yu, S_chai, s_nu = d.collide(g, p, np.full(shape, p.s[9]))
        S = S_yu if drive == "yu" else S_chai
        lhs = s_nu * (3.0 * (p.nu0 + p.c_smag**2 * np.sqrt(2.0 * d.strain_sq(S))) + 0.5)
        assert np.abs(lhs - 1.0).max() < 1e-14
        assert np.abs(S_yu - S_chai).max() <= 1e-13 * np.abs(S_yu).max()
        assert np.abs(d.strain_of_state(g, p, np.full(shape, p.s[9]), drive) - S).max() == 0.0
        p0 = d.Params(visc_kind="smagorinsky_implicit", visc_strain=drive, nu0=0.1, c_smag=0.0)
        assert np.abs(d.collide(g, p0, np.full(shape, p.s[9]))[3] - 1.0 / 0.8).max() < 1e-14


def test_implicit_smagorinsky_conserves():
    shape = (3, 5, 7)
    p = d.Params(visc_kind="smagorinsky_implicit", nu0=0.01, c_smag=0.2)
    u = synth.random_vector(shape, seed=42, scale=0.03)[:3]
    sim = d.Simulation(p, d.init_populations(np.zeros(shape), u, p))
    m0 = sim.g.sum()
    j0 = np.tensordot(d.C.astype(float), sim.g, axes=(1, 0)).reshape(3, -1).sum(1)
    sim.step(20)
    assert abs(sim.g.sum() - m0) < 1e-13
    j1 = np.tensordot(d.C.astype(float), sim.g, axes=(1, 0)).reshape(3, -1).sum(1)
    assert np.abs(j1 - j0).max() < 1e-13


def test_naive_loop_matches_vectorised_step():
    """Brute force: the per-node loop (explicit neighbour indices, the closed-form Yu-type
    formula, an explicit per-node T^-1 diag(s) T) reproduces the vectorised D3Q15 step, with
    walls, a force field and variable viscosity."""
    from oracle import naive_other
    shape = (3, 4, 5)
    for kw in (dict(), dict(visc_kind="smagorinsky", nu0=0.02, c_smag=0.3),
               dict(visc_kind="powerlaw", visc_strain="chai", K_pl=0.02, n_pl=1.4, walls_y=True,
                    force=synth.random_vector(shape, seed=5, scale=1e-3))):
        p = d.Params(**kw)
        g = synth.random_state(15, shape, seed=7, scale=0.01)
        sn = np.full(shape, p.s[9]) * (1 + 0.1 * synth.random_vector(shape, seed=9, scale=1.0)[0])
        g_post, S_yu, S_chai, s_nu = d.collide(g, p, sn)
        nxt = d.stream(g_post, p.walls_y)
        g2, Sy, Sc, snew = naive_other.step(d, g, p, sn)
        assert np.abs(nxt - g2).max() < 1e-15
        assert np.abs(S_yu - Sy).max() < 1e-15
        assert np.abs(S_chai - Sc).max() < 1e-15
        assert np.abs(s_nu - snew).max() < 1e-14


def _ce_residual(N, plane, tau=0.8):
    shape = [1, 1, 1]
    for a in plane:
        shape[2 - a] = N
    shape = tuple(shape)
    u0 = 0.02 * 16 / N
    steps = int(60 * (N / 16) ** 2)
    dr, u, gu = synth.tgv_rotated(shape, u0, 1.0, plane)
    p = d.Params(s=d.default_rates(tau))
    sim = d.Simulation(p, d.init_populations(dr, u, p))
    sim.step(steps)
    k = 2.0 * np.pi / N
    dec = np.exp(-cf.nu_of_rate(1 / tau) * k * k * steps)
    drho, j = d.macroscopic(sim.g)
    mneq = d.moments(sim.g) - d.m_eq(drho, j, p.rho0)
    pred = d.ce_neq_moments(gu * dec, p, float(p.s[9]))
    rows = [1, 9, 10, 11, 12, 13]
    return np.abs(mneq[rows] - pred[rows]).max() / np.abs(pred[rows]).max()


@pytest.mark.slow
@pytest.mark.parametrize("plane", [(0, 1), (1, 2)])
def test_chapman_enskog_prediction_of_the_nonequilibrium_moments(plane):
    """The non-equilibrium moments the Section 5.4 Yu-type formula inverts (ce_neq_moments)
    are what the D3Q15 dynamics produce on a smooth flow: started from the plain equilibrium,
    the measured m - m^eq approaches the prediction from grad u at about second order."""
    e = [_ce_residual(N, plane) for N in (16, 32, 64)]
    assert e[-1] < 5e-3, e
    assert all(np.log2(a / b) > 1.7 for a, b in zip(e[:-1], e[1:])), e
