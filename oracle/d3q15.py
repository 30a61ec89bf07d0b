"""FP64 oracle: D3Q15 MRT step with the Chai strain and the Yu-type formula obtained by the
route of Section 5.4.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 5.3 states that the Chai formula (Eq. ChaiS) holds on D3Q15, and Section 5.4 gives
the procedure for a Yu-type formula on another lattice: put eps m^(1) = m - m^eq in place of
T f^neq, form M = T^-1 Lambda-hat m^(1), N_ab = sum_i c_ia c_ib M_i and
S_ab = -N_ab / (2 rho0 c_s^2 delta_t). The paper gives no D3Q15 matrix; the one used here is
the d'Humieres et al. (2002) basis (outside the paper), written as polynomials of the
velocity c:
  rho 1 | e c^2 - 2 | eps (15 c^4 - 55 c^2 + 32)/2 | j_a c_a | q_a c_a (5 c^2 - 13)/2 |
  3p_xx 2c_x^2 - c_y^2 - c_z^2 | p_ww c_y^2 - c_z^2 | p_xy, p_yz, p_xz c_a c_b | m_xyz c_x c_y c_z
with the rows ordered rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, p_ww, p_xy, p_yz,
p_xz, m_xyz. Velocities: rest, the six faces, the eight corners, opposite pairs adjacent.
Weights 2/9, 1/9, 1/72 (c_s^2 = 1/3). The equilibrium is the paper's delta-rho form of
Eq. edf with these weights and m^eq = T g^eq (as for D2Q9).

State layout (15, nz, ny, nx); strain layout (6, nz, ny, nx) in the order xx, yy, zz, xy,
yz, xz.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

Q = 15
CS2 = 1.0 / 3.0

C = np.array([[0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1],
              [0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1],
              [0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1]], dtype=np.int64)
W = np.array([2.0 / 9.0] + [1.0 / 9.0] * 6 + [1.0 / 72.0] * 8)


def _basis_rows() -> np.ndarray:
    x, y, z = (C[a].astype(np.float64) for a in range(3))
    c2 = x * x + y * y + z * z
    return np.stack([
        np.ones(Q), c2 - 2.0, (15.0 * c2 * c2 - 55.0 * c2 + 32.0) / 2.0,
        x, x * (5.0 * c2 - 13.0) / 2.0, y, y * (5.0 * c2 - 13.0) / 2.0, z, z * (5.0 * c2 - 13.0) / 2.0,
        2.0 * x * x - y * y - z * z, y * y - z * z, x * y, y * z, x * z, x * y * z,
    ])


T = _basis_rows()
TINV = np.linalg.inv(T)
OPP = np.array([int(np.flatnonzero((C == -C[:, i:i + 1]).all(axis=0))[0]) for i in range(Q)])
NU_SLOTS = (9, 10, 11, 12, 13)
_PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2))


def default_rates(tau_nu: float, s_e: float = 1.6, s_eps: float = 1.2, s_q: float = 1.6, s_m: float = 1.2,
                  s_c: float = 0.0) -> np.ndarray:
    """Diagonal of Lambda-hat: conserved rows s_c, e s_e, eps s_eps, q s_q, the five
    second-order rows s_nu = 1/tau_nu, m_xyz s_m. The non-viscous values are the ones
    d'Humieres et al. (2002) suggest for D3Q15 (outside the paper); the strain depends only
    on s_e and s_nu."""
    s_nu = 1.0 / tau_nu
    return np.array([s_c, s_e, s_eps, s_c, s_q, s_c, s_q, s_c, s_q, s_nu, s_nu, s_nu, s_nu, s_nu, s_m])


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
    force: np.ndarray | None = None  # (3,) uniform or (3, nz, ny, nx)
    force_corrected: bool = False  # strain from the force-corrected non-equilibrium part

    def force_field(self, shape) -> np.ndarray:
        if self.force is None:
            return np.zeros((3,) + tuple(shape))
        F = np.asarray(self.force, dtype=np.float64)
        if F.shape == (3,):
            return np.broadcast_to(F.reshape(3, 1, 1, 1), (3,) + tuple(shape)).copy()
        return F.reshape((3,) + tuple(shape))


def _dot_c(v):
    return np.tensordot(C.T.astype(np.float64), v, axes=(1, 0))


def _w(ndim):
    return W.reshape((Q,) + (1,) * ndim)


def g_eq(drho, j, rho0):
    """delta-rho form of Eq. edf with the D3Q15 weights, u = j / rho0."""
    u = j / rho0
    cu = _dot_c(u)
    usq = (u * u).sum(axis=0)
    return _w(drho.ndim) * (drho[None] + rho0 * (cu / CS2 + cu**2 / (2 * CS2**2) - usq[None] / (2 * CS2)))


def m_eq(drho, j, rho0):
    """Equilibrium moments (= T g^eq, pinned by a test): (drho, -drho + |j|^2/rho0,
    drho - 5|j|^2/rho0, j_x, -7j_x/3, j_y, -7j_y/3, j_z, -7j_z/3, (2j_x^2 - j_y^2 - j_z^2)/rho0,
    (j_y^2 - j_z^2)/rho0, j_x j_y/rho0, j_y j_z/rho0, j_x j_z/rho0, 0)."""
    jx, jy, jz = j
    jj = (jx * jx + jy * jy + jz * jz) / rho0
    return np.stack([drho, -drho + jj, drho - 5.0 * jj, jx, -7.0 * jx / 3.0, jy, -7.0 * jy / 3.0, jz,
                     -7.0 * jz / 3.0, (2.0 * jx * jx - jy * jy - jz * jz) / rho0, (jy * jy - jz * jz) / rho0,
                     jx * jy / rho0, jy * jz / rho0, jx * jz / rho0, np.zeros_like(drho)])


def guo_force_populations(j, F, rho0):
    """F-bar = (d g^eq / d j) . F for the delta-rho equilibrium (Guo forcing)."""
    u = j / rho0
    cu, cF = _dot_c(u), _dot_c(F)
    uF = (u * F).sum(axis=0)
    return _w(j.ndim - 1) * (cF / CS2 + cu * cF / CS2**2 - uF[None] / CS2)


def macroscopic(g, F=None):
    drho = g.sum(axis=0)
    j = np.tensordot(C.astype(np.float64), g, axes=(1, 0))
    if F is not None:
        j = j + 0.5 * F
    return drho, j


def moments(g):
    return np.tensordot(T, g, axes=(1, 0))


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
    return m - meq + 0.5 * moments(Fbar), f_neq + 0.5 * Fbar


def strain_chai(f_neq, s, rho0):
    """Eq. ChaiS on D3Q15: -sum_i c_i c_i (T^-1 Lambda-hat T)_ij f_j^neq / (2 rho0 c_s^2)."""
    M = np.tensordot(TINV, _sv(s, f_neq.ndim) * moments(f_neq), axes=(1, 0))
    return _contract_cc(M, rho0)


def strain_yu_type(m_neq, s, rho0):
    """Section 5.4 route: eps m^(1) = m - m^eq in place of T f^neq, M = T^-1 Lambda-hat m^(1),
    N = sum c c M, S = -N / (2 rho0 c_s^2)."""
    M = np.tensordot(TINV, _sv(s, m_neq.ndim) * m_neq, axes=(1, 0))
    return _contract_cc(M, rho0)


def strain_sq(S):
    return S[0] ** 2 + S[1] ** 2 + S[2] ** 2 + 2.0 * (S[3] ** 2 + S[4] ** 2 + S[5] ** 2)


def viscosity_rate(S, p: Params, s_nu_const: float):
    """s_nu = 1/(3 nu + 1/2) from |S| = sqrt(2 S:S), the models of the D3Q19 oracle."""
    shape = S.shape[1:]
    if p.visc_kind == "const":
        return np.full(shape, s_nu_const)
    gamma = np.sqrt(2.0 * strain_sq(S))
    if p.visc_kind == "smagorinsky":
        nu = p.nu0 + p.c_smag**2 * gamma
    elif p.visc_kind == "powerlaw":
        with np.errstate(divide="ignore", invalid="ignore"):
            nu = p.K_pl * np.power(gamma, p.n_pl - 1.0)
        if p.n_pl < 1.0:
            nu = np.where(gamma > 0, nu, p.nu_max)
        elif p.n_pl > 1.0:
            nu = np.where(gamma > 0, nu, p.nu_min)
        else:
            nu = np.full(shape, p.K_pl)
        nu = np.clip(nu, p.nu_min, p.nu_max)
    else:
        raise ValueError(p.visc_kind)
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
    """m* = m - L (m - m^eq) + (I - L/2) T F-bar; g* = T^-1 m* (Eq. mrteqvT on D3Q15), with
    the strains of the incoming state at the lagged s_nu. Returns (g*, S_yu_type, S_chai,
    s_nu)."""
    F = p.force_field(g.shape[1:])
    drho, j = macroscopic(g, F)
    m = moments(g)
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
        s_nu = viscosity_rate(S_yu if p.visc_strain == "yu" else S_chai, p, float(p.s[9]))
    s = rates_field(p, s_nu)
    SF = moments(guo_force_populations(j, F, p.rho0))
    m_post = m - s * (m - meq) + (1.0 - 0.5 * s) * SF
    return np.tensordot(TINV, m_post, axes=(1, 0)), S_yu, S_chai, s_nu


def stream(g_post, walls_y=False):
    """g_i(x + c_i, n+1) = g*_i(x, n), periodic; halfway bounce-back at the y-walls."""
    out = np.empty_like(g_post)
    ny = g_post.shape[2]
    for i in range(Q):
        cx, cy, cz = (int(v) for v in C[:, i])
        out[i] = np.roll(g_post[i], shift=(cz, cy, cx), axis=(0, 1, 2))
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
    mn, fn = strain_nonequilibrium(moments(g), m_eq(drho, j, p.rho0), g - g_eq(drho, j, p.rho0), j, F, p)
    if kind == "yu":
        return strain_yu_type(mn, s, p.rho0)
    return strain_chai(fn, s, p.rho0)


def ce_neq_moments(grad_u, p: Params, s_nu: float):
    """Non-equilibrium moments that make the Yu-type strain equal the symmetric part of
    grad_u (grad_u[a, b] = d u_b / d x_a), every other row zero (the D3Q15 counterpart of
    Eq. YuLuobasis):
      m1 = -2 div j / (3 s_e), m9 = -2 (3 d_x j_x - div j) / (3 s_nu),
      m10 = -2 (d_y j_y - d_z j_z) / (3 s_nu), m11..13 = -(d_a j_b + d_b j_a) / (3 s_nu)."""
    dj = p.rho0 * grad_u
    div = dj[0, 0] + dj[1, 1] + dj[2, 2]
    out = np.zeros((Q,) + grad_u.shape[2:])
    out[1] = -2.0 * div / (3.0 * float(p.s[1]))
    out[9] = -2.0 * (3.0 * dj[0, 0] - div) / (3.0 * s_nu)
    out[10] = -2.0 * (dj[1, 1] - dj[2, 2]) / (3.0 * s_nu)
    out[11] = -(dj[0, 1] + dj[1, 0]) / (3.0 * s_nu)
    out[12] = -(dj[1, 2] + dj[2, 1]) / (3.0 * s_nu)
    out[13] = -(dj[0, 2] + dj[2, 0]) / (3.0 * s_nu)
    return out


def init_populations(drho, u, p: Params, grad_u=None):
    g = g_eq(drho, p.rho0 * u, p.rho0)
    if grad_u is not None:
        g = g + np.tensordot(TINV, ce_neq_moments(grad_u, p, float(p.s[9])), axes=(1, 0))
    return g


def diagnostics(g, p: Params, s_nu) -> dict:
    F = p.force_field(g.shape[1:])
    drho, j = macroscopic(g, F)
    S = strain_of_state(g, p, s_nu, "yu")
    return {
        "mass": float(drho.sum()),
        "mom": j.reshape(3, -1).sum(axis=1),
        "ke": float(((j * j).sum(axis=0) / (2.0 * p.rho0)).sum()),
        "ss": float(strain_sq(S).sum()),
        "umax": float(np.sqrt((j * j).sum(axis=0)).max() / p.rho0),
        "nonfinite": int((~np.isfinite(g)).sum()),
    }


class Simulation:
    def __init__(self, p: Params, g0):
        self.p = p
        self.g = np.array(g0, dtype=np.float64)
        self.s_nu = np.full(self.g.shape[1:], float(p.s[9]))
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

    def diagnostics(self):
        return diagnostics(self.g, self.p, self.s_nu)
