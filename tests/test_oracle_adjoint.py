"""Pins of the FP64 adjoint oracle: transposes checked by dot-product tests against the
pinned forward step, and whole gradients by central finite differences."""
import numpy as np
import pytest

import synth
from oracle import adjoint as adj
from oracle import d3q19 as d


def _fd5(f, h=1.0):
    """Five-point central difference at 0: exact for polynomials of degree <= 4."""
    return (8.0 * (f(h) - f(-h)) - (f(2 * h) - f(-2 * h))) / (12.0 * h)


def _params(tau=0.8):
    return d.Params(s=d.default_rates(tau))


def _state(shape, seed, p):
    u = synth.random_vector(shape, seed=seed, scale=0.03)
    return d.init_populations(np.zeros(shape), u, p) + synth.random_state(19, shape, seed=seed + 1, scale=2e-3)


@pytest.mark.parametrize("walls", [False, True])
def test_stream_transpose(walls):
    """<P v, w> = <v, P^T w> for the periodic and the bounce-back streaming."""
    shape = (3, 5, 4)
    v = synth.random_state(19, shape, seed=1)
    w = synth.random_state(19, shape, seed=2)
    lhs = (d.stream(v, walls) * w).sum()
    rhs = (v * adj.stream_transpose(w, walls)).sum()
    assert abs(lhs - rhs) <= 1e-15 * abs(lhs) + 1e-18


def test_collision_jacobians_are_exact():
    """The collision is quadratic in (g, F): (C(g+v) - C(g-v))/2 = (dC/dg) v exactly, for a
    unit-size v as well, and likewise for F."""
    shape = (2, 3, 4)
    p = _params(0.7)
    g = _state(shape, 3, p)
    F = synth.random_vector(shape, seed=4, scale=1e-4)
    pf = adj._with_force(p, F)
    sn = np.full(shape, p.s[9])
    Jgg, JgF = adj.collision_jacobians(g, F, p)
    v = synth.random_state(19, shape, seed=5, scale=1.0)
    lin = (d.collide(g + v, pf, sn).g_post - d.collide(g - v, pf, sn).g_post) / 2.0
    ref = np.einsum("mil,lm->im", Jgg, v.reshape(19, -1)).reshape(g.shape)
    assert np.abs(lin - ref).max() < 1e-13 * np.abs(ref).max()
    vF = synth.random_vector(shape, seed=6, scale=1.0)
    linF = (d.collide(g, adj._with_force(p, F + vF), sn).g_post - d.collide(g, adj._with_force(p, F - vF), sn).g_post) / 2
    refF = np.einsum("mik,km->im", JgF, vF.reshape(3, -1)).reshape(g.shape)
    assert np.abs(linF - refF).max() < 1e-13 * np.abs(refF).max()


@pytest.mark.parametrize("walls", [False, True])
def test_adjoint_step_dot_product(walls):
    """<L v, w> = <v, L^T w> with L the linearised step (collide + stream), L v taken from
    the forward oracle by an exact central difference."""
    shape = (3, 4, 5)
    p = _params(0.9)
    p.walls_y = walls
    g = _state(shape, 7, p)
    F = synth.random_vector(shape, seed=8, scale=1e-4)
    pf = adj._with_force(p, F)
    sn = np.full(shape, p.s[9])

    def step(gg, FF):
        return d.stream(d.collide(gg, adj._with_force(p, FF), sn).g_post, walls)

    v = synth.random_state(19, shape, seed=9, scale=1e-2)
    vF = synth.random_vector(shape, seed=10, scale=1e-2)
    w = synth.random_state(19, shape, seed=11, scale=1.0)
    Lv = (step(g + v, F) - step(g - v, F)) / 2.0
    LvF = (step(g, F + vF) - step(g, F - vF)) / 2.0
    lam, gF = adj.adjoint_step(w, g, F, pf)
    assert abs((Lv * w).sum() - (v * lam).sum()) <= 1e-13 * abs((Lv * w).sum())
    assert abs((LvF * w).sum() - (vF * gF).sum()) <= 1e-13 * abs((LvF * w).sum())


def test_loss_seed_against_finite_differences():
    shape = (3, 4, 5)
    p = _params(0.8)
    g = _state(shape, 12, p)
    F = synth.random_vector(shape, seed=13, scale=1e-3)
    J, lam, gF = adj.strain_loss_seed(g, F, p)
    assert abs(J - adj.strain_loss(g, F, p)) <= 1e-13 * J
    # J is a polynomial of degree 4 in (g, F): the five-point central difference is exact
    v = synth.random_state(19, shape, seed=14, scale=1e-3)
    vF = synth.random_vector(shape, seed=15, scale=1e-3)
    assert abs(_fd5(lambda t: adj.strain_loss(g + t * v, F, p)) - (lam * v).sum()) <= 1e-10 * abs((lam * v).sum())
    assert abs(_fd5(lambda t: adj.strain_loss(g, F + t * vF, p)) - (gF * vF).sum()) <= 1e-9 * abs((gF * vF).sum())


def test_init_adjoint_dot_product():
    shape = (2, 3, 4)
    p = _params()
    u0 = synth.random_vector(shape, seed=16, scale=0.05)
    lam = synth.random_state(19, shape, seed=17)
    v = synth.random_vector(shape, seed=18, scale=1.0)
    z = np.zeros(shape)
    lin = (d.g_eq(z, p.rho0 * (u0 + v), p.rho0) - d.g_eq(z, p.rho0 * (u0 - v), p.rho0)) / 2.0
    assert abs((lin * lam).sum() - (adj.init_adjoint(lam, u0, p) * v).sum()) <= 1e-13 * abs((lin * lam).sum())


def _c4_problem(n=16, seed_u=1704, seed_f=7559):
    shape = (n, n, n)
    u0 = synth.spectrum_velocity(shape, seed=seed_u, u_rms=0.04)
    F = synth.uniform_random_force(shape, seed=seed_f, amp=1e-6)
    return _params(0.8), u0, F


@pytest.mark.slow
def test_gradient_against_central_differences_16_cubed():
    """The C4 recipe on 16^3 (50 steps, checkpoint every 10): directional derivatives in
    u0 and F, and pointwise entries, against central differences to 1e-6 relative."""
    p, u0, F = _c4_problem()
    nsteps = 50
    J, gu, gF = adj.gradient(u0, F, p, nsteps, every=10)
    assert abs(J - adj.forward(u0, F, p, nsteps)) <= 1e-12 * J
    # fourth-order central differences; steps small against |u0| ~ 0.04 and |F| ~ 1e-6
    du = synth.random_vector(u0.shape[1:], seed=3, scale=1.0)
    fd = _fd5(lambda t: adj.forward(u0 + t * du, F, p, nsteps), h=1e-5)
    assert abs(fd - (gu * du).sum()) <= 1e-6 * abs(fd)
    dF = synth.random_vector(u0.shape[1:], seed=4, scale=1.0)
    fdF = _fd5(lambda t: adj.forward(u0, F + t * dF, p, nsteps), h=1e-8)
    assert abs(fdF - (gF * dF).sum()) <= 1e-6 * abs(fdF)
    for (c, z, y, x) in ((0, 3, 5, 7), (2, 15, 0, 9)):
        e = np.zeros_like(u0)
        e[c, z, y, x] = 1.0
        fdp = _fd5(lambda t: adj.forward(u0 + t * e, F, p, nsteps), h=1e-4)
        assert abs(fdp - gu[c, z, y, x]) <= 1e-6 * np.abs(gu).max()


def test_checkpointing_recomputes_bit_identically():
    p, u0, F = _c4_problem(n=6)
    a = adj.gradient(u0, F, p, 12, every=None)
    b = adj.gradient(u0, F, p, 12, every=5)
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
