"""FP64 oracle: He-Luo D2Q9 MRT step with the Chai strain and the Yu-type formula obtained
by the route of Section 5.4.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper works out D3Q19 only; Section 5.3 states that the Chai formula (Eq. ChaiS)
applies unchanged to D2Q9, and Section 5.4 gives the procedure for a Yu-type formula on
another lattice: replace T f^neq by eps m^(1) = m - m^eq, form M = T^-1 Lambda-hat m^(1),
N_ab = sum_i c_ia c_ib M_i and S_ab = -N_ab / (2 rho0 c_s^2 delta_t). This module does
exactly that. The D2Q9 velocity set, weights and transformation matrix are the common
Lallemand-Luo choice (outside the paper): velocity order 0, E, N, W, S, NE, NW, SW, SE;
moment rows rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy. The equilibrium is the paper's
delta-rho form of Eq. edf with the D2Q9 weights, and m^eq is defined as T g^eq (the D2Q9
counterpart of the D3Q19 choice omega_eps = 3, omega_epsj = -11/2, omega_xx = -1/2).

State layout (9, 1, ny, nx); strain layout (3, 1, ny, nx) in the order xx, yy, xy.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

Q = 9
CS2 = 1.0 / 3.0

C = np.array([[0, 1, 0, -1, 0, 1, -1, -1, 1],
              [0, 0, 1, 0, -1, 1, 1, -1, -1]], dtype=np.int64)
W = np.array([4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4)
T = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
], dtype=np.float64)
TINV = np.linalg.inv(T)
OPP = np.array([int(np.flatnonzero((C == -C[:, i:i + 1]).all(axis=0))[0]) for i in range(Q)])
NU_SLOTS = (7, 8)
_PAIRS = ((0, 0), (1, 1), (0, 1))


def default_rates(tau_nu: float, s_e: float = 1.19, s_eps: float = 1.4, s_q: float = 1.2,
                  s_c: float = 0.0) -> np.ndarray:
    """(s_c, s_e, s_eps, s_c, s_q, s_c, s_q, s_nu, s_nu), s_nu = 1/tau_nu. The non-viscous
    rates (a choice outside the paper) are the ones used for D3Q19; with the often quoted
    s_q = 1.9 the strain still converges but its observed order at N <= 64 drops below 1.8."""
    s_nu = 1.0 / tau_nu
    return np.array([s_c, s_e, s_eps, s_c, s_q, s_c, s_q, s_nu, s_nu])


@dataclass
class Params:
    rho0: float = 1.0
    s: np.ndarray = field(default_factory=lambda: default_rates(0.8))
    visc_kind: str = "const"
    visc_strain: str = "yu"
    nu0: float = 0.0
    c_smag: float = 0.1
    K_pl: float = 0.1
    n_pl: float = 1.0
    nu_min: float = 1e-3
    nu_max: float = 1.0
    walls_y: bool = False
    force: np.ndarray | None = None  # (2,) uniform or (2, 1, ny, nx)
    force_corrected: bool = False  # strain from the force-corrected non-equilibrium part

    def force_field(self, shape) -> np.ndarray:
        if self.force is None:
            return np.zeros((2,) + tuple(shape))
        F = np.asarray(self.force, dtype=np.float64)
        if F.shape == (2,):
            return np.broadcast_to(F.reshape(2, 1, 1, 1), (2,) + tuple(shape)).copy()
        return F.reshape((2,) + tuple(shape))


def _dot_c(v):
    return np.tensordot(C.T.astype(np.float64), v, axes=(1, 0))


def g_eq(drho, j, rho0):
    """delta-rho form of Eq. edf with the D2Q9 weights, u = j / rho0."""
    u = j / rho0
    cu = _dot_c(u)
    usq = (u * u).sum(axis=0)
    return W.reshape((Q,) + (1,) * drho.ndim) * (drho[None] + rho0 * (cu / CS2 + cu**2 / (2 * CS2**2) - usq[None] / (2 * CS2)))


def m_eq(drho, j, rho0):
    """Equilibrium moments of the He-Luo D2Q9 model (= T g^eq, pinned by a test):
    (drho, -2 drho + 3|j|^2/rho0, drho - 3|j|^2/rho0, j_x, -j_x, j_y, -j_y,
     (j_x^2 - j_y^2)/rho0, j_x j_y / rho0)."""
    jx, jy = j
    jj = (jx * jx + jy * jy) / rho0
    return np.stack([drho, -2 * drho + 3 * jj, drho - 3 * jj, jx, -jx, jy, -jy,
                     (jx * jx - jy * jy) / rho0, jx * jy / rho0])


def guo_force_populations(j, F, rho0):
    """(d g^eq / d j) . F for the D2Q9 He-Luo equilibrium (Guo forcing)."""
    u = j / rho0
    cu, cF = _dot_c(u), _dot_c(F)
    uF = (u * F).sum(axis=0)
    return W.reshape((Q,) + (1,) * (j.ndim - 1)) * (cF / CS2 + cu * cF / CS2**2 - uF[None] / CS2)


def macroscopic(g, F=None):
    drho = g.sum(axis=0)
    j = np.tensordot(C.astype(np.float64), g, axes=(1, 0))
    if F is not None:
        j = j + 0.5 * F
    return drho, j


def _contract_cc(M, rho0):
    Cf = C.astype(np.float64)
    return np.stack([-np.tensordot(Cf[a] * Cf[b], M, axes=(0, 0)) / (2.0 * rho0 * CS2) for a, b in _PAIRS])


def _sv(s, ndim):
    return s if s.ndim == ndim else s.reshape((Q,) + (1,) * (ndim - 1))


def strain_nonequilibrium(m, meq, f_neq, j, F, p: Params):
    """(m - m^eq, f - f^eq), or with ``p.force_corrected`` both plus half the Guo source
    (T F-bar / 2 and F-bar / 2): the first-order Chapman-Enskog balance of the forced
    collision, as for D3Q19."""
    if not p.force_corrected:
        return m - meq, f_neq
    Fbar = guo_force_populations(j, F, p.rho0)
    return m - meq + 0.5 * np.tensordot(T, Fbar, axes=(1, 0)), f_neq + 0.5 * Fbar


def strain_chai(f_neq, s, rho0):
    """Eq. ChaiS on D2Q9: -sum_i c_i c_i (T^-1 Lambda-hat T)_ij f_j^neq / (2 rho0 c_s^2)."""
    M = np.tensordot(TINV, _sv(s, f_neq.ndim) * np.tensordot(T, f_neq, axes=(1, 0)), axes=(1, 0))
    return _contract_cc(M, rho0)


def strain_yu_type(m_neq, s, rho0):
    """Section 5.4 route: eps m^(1) = m - m^eq in place of T f^neq, M = T^-1 Lambda-hat m^(1),
    N = sum c c M, S = -N / (2 rho0 c_s^2)."""
    M = np.tensordot(TINV, _sv(s, m_neq.ndim) * m_neq, axes=(1, 0))
    return _contract_cc(M, rho0)


def strain_sq(S):
    return S[0] ** 2 + S[1] ** 2 + 2.0 * S[2] ** 2


def viscosity_rate(S, p: Params, s_nu_const: float):
    """s_nu = 1/(3 nu + 1/2) from |S| = sqrt(2 S:S), as in the D3Q19 oracle."""
    shape = S.shape[1:]
    if p.visc_kind == "const":
        return np.full(shape, s_nu_const)
    gamma = np.sqrt(2.0 * strain_sq(S))
    if p.visc_kind == "smagorinsky":
        nu = p.nu0 + p.c_smag**2 * gamma
    else:
        with np.errstate(divide="ignore", invalid="ignore"):
            nu = p.K_pl * np.power(gamma, p.n_pl - 1.0)
        if p.n_pl < 1.0:
            nu = np.where(gamma > 0, nu, p.nu_max)
        elif p.n_pl > 1.0:
            nu = np.where(gamma > 0, nu, p.nu_min)
        else:
            nu = np.full(shape, p.K_pl)
        nu = np.clip(nu, p.nu_min, p.nu_max)
    return 1.0 / (3.0 * nu + 0.5)


def implicit_smagorinsky_rate(S_of_s, p: Params, shape):
    """s_nu solving s = 1 / (3 (nu0 + C_s^2 |S(s)|) + 1/2) per node, S(s) being the strain
    formula at s_nu = s. The Yu-type formula is affine in s_nu with an isotropic s_e part and a
    traceless s_nu part, so |S(s)| increases with s and the root in (0, 2] is unique: plain
    bisection to FP64 resolution."""
    lo = np.zeros(shape)
    hi = np.full(shape, 2.0)
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        nu = p.nu0 + p.c_smag**2 * np.sqrt(2.0 * strain_sq(S_of_s(mid)))
        f = mid * (3.0 * nu + 0.5) - 1.0
        lo = np.where(f < 0.0, mid, lo)
        hi = np.where(f < 0.0, hi, mid)
    return 0.5 * (lo + hi)


def rates_field(p: Params, s_nu):
    s = np.broadcast_to(p.s.reshape((Q,) + (1,) * s_nu.ndim), (Q,) + s_nu.shape).copy()
    for k in NU_SLOTS:
        s[k] = s_nu
    return s


def collide(g, p: Params, s_nu_prev):
    """m* = m - L (m - m^eq) + (I - L/2) T F-bar; g* = T^-1 m*. Returns
    (g*, S_yu_type, S_chai, s_nu) with the strains of the incoming state."""
    F = p.force_field(g.shape[1:])
    drho, j = macroscopic(g, F)
    m = np.tensordot(T, g, axes=(1, 0))
    meq = m_eq(drho, j, p.rho0)
    mn, fn = strain_nonequilibrium(m, meq, g - g_eq(drho, j, p.rho0), j, F, p)
    if p.visc_kind == "smagorinsky_implicit":
        # non-lagged coupling: the strain uses the rate of this very collision
        def yu_of(sv):
            return strain_yu_type(mn, rates_field(p, sv), p.rho0)

        def chai_of(sv):
            return strain_chai(fn, rates_field(p, sv), p.rho0)

        s_nu = implicit_smagorinsky_rate(yu_of if p.visc_strain == "yu" else chai_of, p, g.shape[1:])
        S_yu, S_chai = yu_of(s_nu), chai_of(s_nu)
    else:
        sp = rates_field(p, s_nu_prev)
        S_yu = strain_yu_type(mn, sp, p.rho0)
        S_chai = strain_chai(fn, sp, p.rho0)
        s_nu = viscosity_rate(S_yu if p.visc_strain == "yu" else S_chai, p, float(p.s[7]))
    s = rates_field(p, s_nu)
    SF = np.tensordot(T, guo_force_populations(j, F, p.rho0), axes=(1, 0))
    m_post = m - s * (m - meq) + (1.0 - 0.5 * s) * SF
    return np.tensordot(TINV, m_post, axes=(1, 0)), S_yu, S_chai, s_nu


def stream(g_post, walls_y=False):
    """g_i(x + c_i, n+1) = g*_i(x, n), periodic; halfway bounce-back at the y-walls."""
    out = np.empty_like(g_post)
    ny = g_post.shape[2]
    for i in range(Q):
        cx, cy = int(C[0, i]), int(C[1, i])
        out[i] = np.roll(g_post[i], shift=(cy, cx), axis=(1, 2))
    if walls_y:
        for i in range(Q):
            cy = int(C[1, i])
            if cy == 1:
                out[i][:, 0, :] = g_post[OPP[i]][:, 0, :]
            elif cy == -1:
                out[i][:, ny - 1, :] = g_post[OPP[i]][:, ny - 1, :]
    return out


def strain_of_state(g, p: Params, s_nu, kind="yu"):
    if p.visc_kind == "smagorinsky_implicit":
        _, S_yu, S_chai, _ = collide(g, p, s_nu)
        return S_yu if kind == "yu" else S_chai
    F = p.force_field(g.shape[1:])
    drho, j = macroscopic(g, F)
    s = rates_field(p, s_nu)
    mn, fn = strain_nonequilibrium(np.tensordot(T, g, axes=(1, 0)), m_eq(drho, j, p.rho0), g - g_eq(drho, j, p.rho0),
                                   j, F, p)
    if kind == "yu":
        return strain_yu_type(mn, s, p.rho0)
    return strain_chai(fn, s, p.rho0)


def ce_neq_moments(grad_u, p: Params, s_nu: float):
    """Chapman-Enskog non-equilibrium moments for D2Q9, the inverse of the Yu-type formula
    (grad_u[a, b] = d u_b / d x_a, a, b in x, y):
    m1 = -2 div j / s_e, m7 = -2 (d_x j_x - d_y j_y) / (3 s_nu), m8 = -(d_x j_y + d_y j_x) / (3 s_nu)."""
    dj = p.rho0 * grad_u
    out = np.zeros((Q,) + grad_u.shape[2:])
    out[1] = -2.0 * (dj[0, 0] + dj[1, 1]) / float(p.s[1])
    out[7] = -2.0 * (dj[0, 0] - dj[1, 1]) / (3.0 * s_nu)
    out[8] = -(dj[0, 1] + dj[1, 0]) / (3.0 * s_nu)
    return out


def init_populations(drho, u, p: Params, grad_u=None):
    g = g_eq(drho, p.rho0 * u, p.rho0)
    if grad_u is not None:
        g = g + np.tensordot(TINV, ce_neq_moments(grad_u, p, float(p.s[7])), axes=(1, 0))
    return g


class Simulation:
    def __init__(self, p: Params, g0):
        self.p = p
        self.g = np.array(g0, dtype=np.float64)
        self.s_nu = np.full(self.g.shape[1:], float(p.s[7]))
        self.last = None

    def step(self, nsteps=1):
        for _ in range(nsteps):
            g_post, Sy, Sc, sn = collide(self.g, self.p, self.s_nu)
            self.g = stream(g_post, self.p.walls_y)
            self.s_nu = sn
            self.last = (Sy, Sc)
        return self.last

    def strain(self, kind="yu"):
        return strain_of_state(self.g, self.p, self.s_nu, kind)
