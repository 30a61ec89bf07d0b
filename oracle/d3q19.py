"""FP64 oracle: He-Luo D3Q19 MRT lattice Boltzmann step and the Yu / Chai strain rates.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never imports this.

State convention. The paper's delta-rho form of the equilibrium (Section 2, the second
Eq. edf) replaces rho by the fluctuation delta_rho = rho - rho_0 to limit round-off. The
oracle stores the matching population deviation g_i = f_i - omega_i rho_0, so that
sum_i g_i = delta_rho and sum_i c_i g_i = j. Every array of populations has shape
(19, nz, ny, nx) with x fastest; velocity-like fields have shape (3, nz, ny, nx); strain
fields have shape (6, nz, ny, nx) in the component order xx, yy, zz, xy, yz, xz.

Lattice units: delta_x = delta_t = c = 1, c_s^2 = 1/3 (Section 2, after Eq. HeLuoD3Q19).

Readings of passages the paper leaves open or prints garbled (each is listed in the
repository's design notes):
* Eq. meq prints the labels of 3 pi_xx^eq and p_ww^eq swapped; the equilibrium moment
  column of Eq. solvem (the d/dt1 vector) fixes m_9..m_12, and that is what ``m_eq`` uses.
* The rates s_e, s_eps, s_q, s_pi, s_t are not given (Eq. sD3Q15meaning); ``default_rates``
  uses the commonly quoted d'Humieres set and s_c = 0 (Section 2 says the conserved rates
  are set to zero).
* With a variable viscosity the strain at step n is evaluated with the s_nu of the previous
  collision at the same node (lagged), held in an explicit field; the
  "smagorinsky_implicit" model instead solves the local coupling s_nu(S(s_nu)) per node.
* Body force: Guo forcing written in moment space, with j = sum c g + F/2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

Q = 19
CS2 = 1.0 / 3.0  # c_s^2 with c = 1 (Section 2)

# Discrete velocities c_0..c_18, Eq. HeLuoD3Q19 (rows: x, y, z).
C = np.array(
    [
        [0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0],
        [0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1],
        [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1],
    ],
    dtype=np.int64,
)

# Weights omega_i, Eq. omega.
W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)

# Transformation matrix T of Section 2 (d'Humieres D3Q19 basis), row by row as printed.
T = np.array(
    [
        [1] * 19,
        [-30, -11, -11, -11, -11, -11, -11, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8],
        [12, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1],
        [0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0],
        [0, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0],
        [0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1],
        [0, 0, 0, -4, 4, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1],
        [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1],
        [0, 0, 0, 0, 0, -4, 4, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1],
        [0, 2, 2, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2],
        [0, -4, -4, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2],
        [0, 0, 0, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0],
        [0, 0, 0, -2, -2, 2, 2, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0],
        [0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0],
        [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1],
        [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0],
        [0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1, 0, 0, 0, 0],
        [0, 0, 0, 0, 0, 0, 0, -1, -1, 1, 1, 0, 0, 0, 0, 1, -1, 1, -1],
        [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1],
    ],
    dtype=np.float64,
)
# T^-1 as a library inverse (Section 2 only states that T is invertible).
TINV = np.linalg.inv(T)

# Index of the opposite velocity, c_opp(i) = -c_i (used only by bounce-back walls).
OPP = np.array([int(np.flatnonzero((C == -C[:, i : i + 1]).all(axis=0))[0]) for i in range(Q)])

# Strain component order used by every strain array.
STRAIN_COMPONENTS = ("xx", "yy", "zz", "xy", "yz", "xz")
_PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2))


def default_rates(tau_nu: float, s_e: float = 1.19, s_eps: float = 1.4, s_q: float = 1.2,
                  s_pi: float = 1.4, s_t: float = 1.98, s_c: float = 0.0) -> np.ndarray:
    """Diagonal of Lambda-hat in the layout of Eq. sD3Q15meaning.

    (s_c, s_e, s_eps, s_c, s_q, s_c, s_q, s_c, s_q, s_nu, s_pi, s_nu, s_pi, s_nu, s_nu,
    s_nu, s_t, s_t, s_t) with s_nu = 1/tau_nu. Section 2 leaves the non-viscous rates open;
    the defaults are the widely used d'Humieres values (a reading, not the paper's).
    """
    s_nu = 1.0 / tau_nu
    return np.array([s_c, s_e, s_eps, s_c, s_q, s_c, s_q, s_c, s_q,
                     s_nu, s_pi, s_nu, s_pi, s_nu, s_nu, s_nu, s_t, s_t, s_t], dtype=np.float64)


NU_SLOTS = (9, 11, 13, 14, 15)  # rows relaxed with s_nu (Eq. sD3Q15meaning)


@dataclass
class Params:
    """Everything one step needs. ``s`` is the diagonal of Lambda-hat (Eq. sD3Q15)."""

    rho0: float = 1.0
    s: np.ndarray = field(default_factory=lambda: default_rates(0.8))
    omega_eps: float = 3.0       # Eq. meq
    omega_epsj: float = -5.5     # Eq. meq
    omega_xx: float = -0.5       # Eq. meq
    visc_kind: str = "const"     # "const" | "smagorinsky" | "powerlaw" | "smagorinsky_implicit"
    visc_strain: str = "yu"      # which formula drives the viscosity: "yu" | "chai"
    nu0: float = 0.0             # Smagorinsky molecular viscosity
    c_smag: float = 0.1          # Smagorinsky constant, filter width Delta = 1
    K_pl: float = 0.1            # power-law consistency
    n_pl: float = 1.0            # power-law index
    nu_min: float = 1e-3
    nu_max: float = 1.0
    walls_y: bool = False        # halfway bounce-back at y = -1/2 and y = ny - 1/2
    force: np.ndarray | None = None  # (3,) uniform or (3, nz, ny, nx) field
    force_corrected: bool = False  # strain from the force-corrected non-equilibrium part

    def force_field(self, shape) -> np.ndarray:
        if self.force is None:
            return np.zeros((3,) + tuple(shape))
        F = np.asarray(self.force, dtype=np.float64)
        if F.shape == (3,):
            return np.broadcast_to(F.reshape(3, 1, 1, 1), (3,) + tuple(shape)).copy()
        return F.reshape((3,) + tuple(shape)).astype(np.float64)


# ---------------------------------------------------------------------------------------
# Equilibria (Section 2)
# ---------------------------------------------------------------------------------------

def _dot_c(v: np.ndarray) -> np.ndarray:
    """(c_i . v) for every i: (3, ...) -> (19, ...)."""
    return np.tensordot(C.T.astype(np.float64), v, axes=(1, 0))


def g_eq(drho: np.ndarray, j: np.ndarray, rho0: float) -> np.ndarray:
    """Equilibrium deviation g_i^eq, the delta-rho form of Eq. edf with u = j / rho_0.

    g_i^eq = omega_i [ delta_rho + rho_0 ( c_i.u / c_s^2 + (c_i.u)^2 / (2 c_s^4)
                                           - |u|^2 / (2 c_s^2) ) ]
    """
    u = j / rho0
    cu = _dot_c(u)
    usq = (u * u).sum(axis=0)
    wshape = (Q,) + (1,) * drho.ndim
    return W.reshape(wshape) * (drho[None] + rho0 * (cu / CS2 + cu**2 / (2 * CS2**2) - usq[None] / (2 * CS2)))


def m_eq(drho: np.ndarray, j: np.ndarray, rho0: float, omega_eps: float = 3.0,
         omega_epsj: float = -5.5, omega_xx: float = -0.5) -> np.ndarray:
    """Equilibrium moments, Eq. meq (rows 9..12 as in the d/dt1 column of Eq. solvem).

    m^eq = (drho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww, pi_ww,
            p_xy, p_yz, p_xz, t_x, t_y, t_z)^eq
    """
    jx, jy, jz = j
    jj = jx * jx + jy * jy + jz * jz
    zero = np.zeros_like(drho)
    pxx3 = (2 * jx * jx - jy * jy - jz * jz) / rho0
    pww = (jy * jy - jz * jz) / rho0
    return np.stack([
        drho,
        -11.0 * drho + 19.0 * jj / rho0,
        omega_eps * drho + omega_epsj * jj / rho0,
        jx, -2.0 * jx / 3.0,
        jy, -2.0 * jy / 3.0,
        jz, -2.0 * jz / 3.0,
        pxx3, omega_xx * pxx3,
        pww, omega_xx * pww,
        jx * jy / rho0, jy * jz / rho0, jx * jz / rho0,
        zero, zero, zero,
    ])


def guo_force_populations(j: np.ndarray, F: np.ndarray, rho0: float) -> np.ndarray:
    """Guo forcing term in velocity space for the He-Luo equilibrium.

    F-bar_i = (d g_i^eq / d j) . F = omega_i [ c_i.F / c_s^2 + (c_i.u)(c_i.F) / c_s^4
                                                - u.F / c_s^2 ],  u = j / rho_0.
    The paper only cites a force-corrected scheme; this is the standard Guo choice
    (a reading), applied in moment space as (I - Lambda-hat/2) T F-bar.
    """
    u = j / rho0
    cu = _dot_c(u)
    cF = _dot_c(F)
    uF = (u * F).sum(axis=0)
    wshape = (Q,) + (1,) * (j.ndim - 1)
    return W.reshape(wshape) * (cF / CS2 + cu * cF / CS2**2 - uF[None] / CS2)


# ---------------------------------------------------------------------------------------
# Macroscopic moments and the two strain formulas (Section 3)
# ---------------------------------------------------------------------------------------

def macroscopic(g: np.ndarray, F: np.ndarray | None = None):
    """delta_rho = sum_i g_i, j = sum_i c_i g_i (+ F/2 with a body force)."""
    drho = g.sum(axis=0)
    j = np.tensordot(C.astype(np.float64), g, axes=(1, 0))
    if F is not None:
        j = j + 0.5 * F
    return drho, j


def moments(g: np.ndarray) -> np.ndarray:
    """m = T |g>, the dense 19x19 product of Section 2."""
    return np.tensordot(T, g, axes=(1, 0))


def strain_yu(m_neq: np.ndarray, s1, s9, rho0: float) -> np.ndarray:
    """Yu formula, Eq. LuoS, with eps m^(1) taken as m - m^eq and delta_t = 1.

    S_xx = -(s1 m1 + 19 s9 m9) / (38 rho0)
    S_yy,zz = -[2 s1 m1 - 19 s9 (m9 -/+ 3 m11)] / (76 rho0)
    S_xy,yz,zx = -3 s9 m13,14,15 / (2 rho0)
    """
    m1, m9, m11 = m_neq[1], m_neq[9], m_neq[11]
    Sxx = -(s1 * m1 + 19.0 * s9 * m9) / (38.0 * rho0)
    Syy = -(2.0 * s1 * m1 - 19.0 * s9 * (m9 - 3.0 * m11)) / (76.0 * rho0)
    Szz = -(2.0 * s1 * m1 - 19.0 * s9 * (m9 + 3.0 * m11)) / (76.0 * rho0)
    Sxy = -3.0 * s9 * m_neq[13] / (2.0 * rho0)
    Syz = -3.0 * s9 * m_neq[14] / (2.0 * rho0)
    Sxz = -3.0 * s9 * m_neq[15] / (2.0 * rho0)
    return np.stack([Sxx, Syy, Szz, Sxy, Syz, Sxz])


def strain_nonequilibrium(m: np.ndarray, meq: np.ndarray, f_neq: np.ndarray, j: np.ndarray, F: np.ndarray,
                          p: Params):
    """The non-equilibrium parts the two strain formulas take: (m - m^eq, f - f^eq), or, with
    ``p.force_corrected``, (m - m^eq + T F-bar / 2, f - f^eq + F-bar / 2).

    The correction (the force effect the paper attributes to Premnath et al., Section 1)
    follows from the first-order Chapman-Enskog balance of the Guo-forced collision:
    s_k (m_k^(1) + S_F,k / 2) equals the force-free gradient term, so the half source added
    to the non-equilibrium moments removes the u F terms that the force puts into the
    second-order moments. Both formulas get the same half source (in moment and in velocity
    space), so their identity (Section 5.1) is kept."""
    if not p.force_corrected:
        return m - meq, f_neq
    Fbar = guo_force_populations(j, F, p.rho0)
    return m - meq + 0.5 * moments(Fbar), f_neq + 0.5 * Fbar


def strain_chai(f_neq: np.ndarray, s: np.ndarray, rho0: float) -> np.ndarray:
    """Chai formula, Eq. ChaiS, with delta_t = 1.

    S = - sum_i c_i c_i (T^-1 Lambda-hat T)_ij f_j^neq / (2 rho0 c_s^2).

    ``s`` is the diagonal of Lambda-hat, either (19,) or (19, ...) per node. The product
    (T^-1 Lambda-hat T) f^neq is formed in the order the paper describes for this formula
    (efficiency subsection): T f^neq, then Lambda-hat, then T^-1, then the c c sum.
    """
    sv = s if s.ndim == f_neq.ndim else s.reshape((Q,) + (1,) * (f_neq.ndim - 1))
    M = np.tensordot(TINV, sv * np.tensordot(T, f_neq, axes=(1, 0)), axes=(1, 0))
    Cf = C.astype(np.float64)
    out = []
    for a, b in _PAIRS:
        N_ab = np.tensordot(Cf[a] * Cf[b], M, axes=(0, 0))
        out.append(-N_ab / (2.0 * rho0 * CS2))
    return np.stack(out)


def strain_norm(S: np.ndarray) -> np.ndarray:
    """|S| = sqrt(2 S:S) with S symmetric (off-diagonal components counted twice)."""
    SS = S[0] ** 2 + S[1] ** 2 + S[2] ** 2 + 2.0 * (S[3] ** 2 + S[4] ** 2 + S[5] ** 2)
    return np.sqrt(2.0 * SS)


def strain_sq(S: np.ndarray) -> np.ndarray:
    """S:S = sum_ab S_ab S_ab (off-diagonal components counted twice)."""
    return S[0] ** 2 + S[1] ** 2 + S[2] ** 2 + 2.0 * (S[3] ** 2 + S[4] ** 2 + S[5] ** 2)


# ---------------------------------------------------------------------------------------
# Viscosity models driven by the strain
# ---------------------------------------------------------------------------------------

def viscosity_rate(S: np.ndarray, p: Params, s_nu_const: float) -> np.ndarray:
    """New s_nu per node: s_nu = 1 / (3 nu + 1/2), nu from the strain magnitude.

    const       : s_nu = s_nu_const everywhere
    smagorinsky : nu = nu0 + (C_s Delta)^2 |S|, Delta = 1
    powerlaw    : nu = clamp(K gamma^(n-1), nu_min, nu_max), gamma = |S|; at gamma = 0
                  nu = nu_max for n < 1, nu_min for n > 1, K for n = 1 (clamped)
    """
    shape = S.shape[1:]
    if p.visc_kind == "const":
        return np.full(shape, s_nu_const)
    gamma = strain_norm(S)
    if p.visc_kind == "smagorinsky":
        nu = p.nu0 + (p.c_smag**2) * gamma
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


def implicit_smagorinsky_rate(S_of_s, p: Params, shape) -> np.ndarray:
    """s_nu solving s = 1 / (3 (nu0 + C_s^2 |S(s)|) + 1/2) at every node, where S(s) is the
    strain formula evaluated with s_nu = s (both formulas are affine in s_nu).

    The s_e part of S is isotropic and the s_nu part traceless, so |S(s)|^2 = |P|^2 + s^2 |A|^2
    and f(s) = s (3 nu(s) + 1/2) - 1 is increasing on [0, 2], with f(0) = -1 and f(2) >= 0:
    the root is unique; plain bisection to FP64 resolution.
    """
    lo = np.zeros(shape)
    hi = np.full(shape, 2.0)
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        nu = p.nu0 + p.c_smag**2 * strain_norm(S_of_s(mid))
        f = mid * (3.0 * nu + 0.5) - 1.0
        lo = np.where(f < 0.0, mid, lo)
        hi = np.where(f < 0.0, hi, mid)
    return 0.5 * (lo + hi)


# ---------------------------------------------------------------------------------------
# Collision, streaming, the step (Eqs. mrteq, mrteqvT)
# ---------------------------------------------------------------------------------------

def rates_field(p: Params, s_nu: np.ndarray) -> np.ndarray:
    """Diagonal of Lambda-hat at every node: p.s with the s_nu slots replaced."""
    s = np.broadcast_to(p.s.reshape((Q,) + (1,) * s_nu.ndim), (Q,) + s_nu.shape).copy()
    for k in NU_SLOTS:
        s[k] = s_nu
    return s


@dataclass
class CollideOut:
    g_post: np.ndarray   # post-collision populations g*(x, n)
    S_yu: np.ndarray     # strain of the pre-collision state, Yu formula
    S_chai: np.ndarray   # strain of the pre-collision state, Chai formula
    s_nu: np.ndarray     # s_nu used in this collision (the lagged value for step n+1)
    drho: np.ndarray
    j: np.ndarray


def collide(g: np.ndarray, p: Params, s_nu_prev: np.ndarray) -> CollideOut:
    """One collision, Eq. mrteqvT in moment space, with the strain of the incoming state.

    m* = m - Lambda-hat (m - m^eq) + (I - Lambda-hat / 2) T F-bar ;  g* = T^-1 m*.
    Both strains use the rates of the previous collision (``s_nu_prev``); the new s_nu
    comes from the strain chosen by ``p.visc_strain`` and relaxes this collision.
    """
    shape = g.shape[1:]
    F = p.force_field(shape)
    drho, j = macroscopic(g, F)
    m = moments(g)
    meq = m_eq(drho, j, p.rho0, p.omega_eps, p.omega_epsj, p.omega_xx)
    mn, fn = strain_nonequilibrium(m, meq, g - g_eq(drho, j, p.rho0), j, F, p)
    if p.visc_kind == "smagorinsky_implicit":
        # non-lagged coupling: the strain uses the rate of this very collision
        def yu_of(sv):
            return strain_yu(mn, float(p.s[1]), sv, p.rho0)

        def chai_of(sv):
            return strain_chai(fn, rates_field(p, sv), p.rho0)

        s_nu = implicit_smagorinsky_rate(yu_of if p.visc_strain == "yu" else chai_of, p, shape)
        S_yu, S_chai = yu_of(s_nu), chai_of(s_nu)
    else:
        s_prev = rates_field(p, s_nu_prev)
        S_yu = strain_yu(mn, s_prev[1], s_prev[9], p.rho0)
        S_chai = strain_chai(fn, s_prev, p.rho0)
        S_drive = S_yu if p.visc_strain == "yu" else S_chai
        s_nu = viscosity_rate(S_drive, p, float(p.s[9]))
    s = rates_field(p, s_nu)
    SF = moments(guo_force_populations(j, F, p.rho0))
    m_post = m - s * (m - meq) + (1.0 - 0.5 * s) * SF
    g_post = np.tensordot(TINV, m_post, axes=(1, 0))
    return CollideOut(g_post, S_yu, S_chai, s_nu, drho, j)


def stream(g_post: np.ndarray, walls_y: bool = False) -> np.ndarray:
    """Streaming, the left side of Eq. mrteq: g_i(x + c_i, n+1) = g*_i(x, n), periodic.

    With ``walls_y`` the links that leave the box through y = -1/2 or y = ny - 1/2 are
    reflected by halfway bounce-back: g_opp(i)(x, n+1) = g*_i(x, n).
    """
    out = np.empty_like(g_post)
    ny = g_post.shape[2]
    for i in range(Q):
        cx, cy, cz = (int(v) for v in C[:, i])
        out[i] = np.roll(g_post[i], shift=(cz, cy, cx), axis=(0, 1, 2))
    if walls_y:
        for i in range(Q):
            cy = int(C[1, i])
            if cy == 1:      # arrivals at y = 0 came through the lower wall
                out[i][:, 0, :] = g_post[OPP[i]][:, 0, :]
            elif cy == -1:   # arrivals at y = ny-1 came through the upper wall
                out[i][:, ny - 1, :] = g_post[OPP[i]][:, ny - 1, :]
    return out


def strain_of_state(g: np.ndarray, p: Params, s_nu: np.ndarray, kind: str = "yu") -> np.ndarray:
    """Strain of a pre-collision state g(x, n) with the rates in ``s_nu`` (Yu or Chai); with
    the implicit Smagorinsky coupling the rate is solved from the state itself."""
    if p.visc_kind == "smagorinsky_implicit":
        out = collide(g, p, s_nu)
        return out.S_yu if kind == "yu" else out.S_chai
    F = p.force_field(g.shape[1:])
    drho, j = macroscopic(g, F)
    s = rates_field(p, s_nu)
    meq = m_eq(drho, j, p.rho0, p.omega_eps, p.omega_epsj, p.omega_xx)
    mn, fn = strain_nonequilibrium(moments(g), meq, g - g_eq(drho, j, p.rho0), j, F, p)
    if kind == "yu":
        return strain_yu(mn, s[1], s[9], p.rho0)
    return strain_chai(fn, s, p.rho0)


# ---------------------------------------------------------------------------------------
# Initial conditions
# ---------------------------------------------------------------------------------------

def ce_neq_moments(grad_u: np.ndarray, p: Params, s_nu: float) -> np.ndarray:
    """Non-equilibrium moments predicted by the Chapman-Enskog analysis, Eq. YuLuobasis.

    grad_u[a, b] = d u_b / d x_a, shape (3, 3, ...). With j = rho0 u and delta_t = 1:
      eps m1  = -38 div j / (3 s1)
      eps m9  = -2 (3 d_x j_x - div j) / (3 s9),  eps m11 = -2 (d_y j_y - d_z j_z) / (3 s9)
      eps m13 = -(d_x j_y + d_y j_x) / (3 s9), m14 (yz), m15 (zx) likewise.
    Every other non-equilibrium moment is set to zero (a reading: the paper derives only
    these rows).
    """
    r = p.rho0
    s1 = float(p.s[1])
    dj = r * grad_u
    div = dj[0, 0] + dj[1, 1] + dj[2, 2]
    out = np.zeros((Q,) + grad_u.shape[2:])
    out[1] = -38.0 * div / (3.0 * s1)
    out[9] = -2.0 * (3.0 * dj[0, 0] - div) / (3.0 * s_nu)
    out[11] = -2.0 * (dj[1, 1] - dj[2, 2]) / (3.0 * s_nu)
    out[13] = -(dj[0, 1] + dj[1, 0]) / (3.0 * s_nu)
    out[14] = -(dj[1, 2] + dj[2, 1]) / (3.0 * s_nu)
    out[15] = -(dj[0, 2] + dj[2, 0]) / (3.0 * s_nu)
    return out


def init_populations(drho: np.ndarray, u: np.ndarray, p: Params,
                     grad_u: np.ndarray | None = None) -> np.ndarray:
    """g(x, 0) = g^eq(delta_rho, rho0 u) [+ T^-1 m^neq from the CE relations if grad_u]."""
    g = g_eq(drho, p.rho0 * u, p.rho0)
    if grad_u is not None:
        g = g + np.tensordot(TINV, ce_neq_moments(grad_u, p, float(p.s[9])), axes=(1, 0))
    return g


# ---------------------------------------------------------------------------------------
# Diagnostics (conservation, Section 4.1 continuity and momentum equations)
# ---------------------------------------------------------------------------------------

def diagnostics(g: np.ndarray, p: Params, s_nu: np.ndarray) -> dict:
    """Global sums of the pre-collision state.

    mass = sum delta_rho; mom = sum (sum_i c_i g_i + F/2); ke = sum |j|^2 / (2 rho0);
    ss = sum S:S (Yu); umax = max |j| / rho0; nonfinite = count of non-finite g.
    """
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
    """A D3Q19 run held as the pre-collision state g(x, n) plus the lagged s_nu field."""

    def __init__(self, p: Params, g0: np.ndarray):
        self.p = p
        self.g = np.array(g0, dtype=np.float64)
        self.s_nu = np.full(self.g.shape[1:], float(p.s[9]))
        self.n = 0
        self.last: CollideOut | None = None

    def step(self, nsteps: int = 1) -> CollideOut:
        for _ in range(nsteps):
            out = collide(self.g, self.p, self.s_nu)
            self.g = stream(out.g_post, self.p.walls_y)
            self.s_nu = out.s_nu
            self.n += 1
            self.last = out
        return self.last

    def strain(self, kind: str = "yu") -> np.ndarray:
        return strain_of_state(self.g, self.p, self.s_nu, kind)

    def diagnostics(self) -> dict:
        return diagnostics(self.g, self.p, self.s_nu)
