"""Exact incompressible Navier-Stokes solutions used as expected values.

TEST INFRASTRUCTURE ONLY. These are textbook closed forms, not the paper's arithmetic; the
paper's claim they serve is that the strain from either formula is second-order accurate
in space (Section 5.1, last paragraph). Node coordinates are the integers 0..N-1 of a
periodic box of N nodes, so kappa = 2 pi / N. Viscosity in lattice units is
nu = (1/s_nu - 1/2) / 3.
"""
from __future__ import annotations

import numpy as np


def nu_of_rate(s_nu: float) -> float:
    return (1.0 / s_nu - 0.5) / 3.0


def _coords(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (x.astype(np.float64), y.astype(np.float64), z.astype(np.float64))


def tgv_rotated_strain(shape, u0: float, nu: float, t: float, plane=(0, 1)) -> np.ndarray:
    """Strain of u_a = u0 sin(k x_b), u_b = u0 sin(k x_a) (Taylor-Green turned by 45 deg).

    The flow decays as exp(-nu k^2 t); S_ab = (u0 k / 2)(cos k x_a + cos k x_b) e^(-nu k^2 t),
    every other component is zero. Returns (6, nz, ny, nx) in order xx, yy, zz, xy, yz, xz.
    """
    a, b = plane
    X = _coords(shape)
    N = shape[2 - a]
    k = 2.0 * np.pi / N
    dec = np.exp(-nu * k * k * t)
    S = np.zeros((6,) + tuple(shape))
    comp = {(0, 1): 3, (1, 2): 4, (0, 2): 5}[tuple(sorted((a, b)))]
    S[comp] = 0.5 * u0 * k * (np.cos(k * X[a]) + np.cos(k * X[b])) * dec
    return S


def tgv_axis_strain(shape, u0: float, nu: float, t: float, plane=(0, 1)) -> np.ndarray:
    """Strain of u_a = u0 sin(k x_a) cos(k x_b), u_b = -u0 cos(k x_a) sin(k x_b).

    Decay exp(-2 nu k^2 t); S_aa = -S_bb = u0 k cos(k x_a) cos(k x_b) e^(-2 nu k^2 t) and
    S_ab = 0 identically.
    """
    a, b = plane
    X = _coords(shape)
    N = shape[2 - a]
    k = 2.0 * np.pi / N
    dec = np.exp(-2.0 * nu * k * k * t)
    S = np.zeros((6,) + tuple(shape))
    val = u0 * k * np.cos(k * X[a]) * np.cos(k * X[b]) * dec
    S[a] = val
    S[b] = -val
    return S


def powerlaw_poiseuille(eta: np.ndarray, H: float, F: float, K: float, n: float) -> np.ndarray:
    """Steady plane Poiseuille velocity of a power-law fluid between walls at eta = 0 and H.

    Stress balance tau(eta) = F (H/2 - eta) with tau = K |du/deta|^(n-1) du/deta
    (kinematic units, rho0 = 1) gives
      u(eta) = n/(n+1) (F/K)^(1/n) [ (H/2)^((n+1)/n) - |eta - H/2|^((n+1)/n) ].
    """
    e = (n + 1.0) / n
    return n / (n + 1.0) * (F / K) ** (1.0 / n) * ((H / 2.0) ** e - np.abs(eta - H / 2.0) ** e)


def startup_poiseuille(eta: np.ndarray, H: float, F: float, nu: float, t: float,
                       terms: int = 2000) -> np.ndarray:
    """Start-up of Newtonian plane Poiseuille flow from rest (odd-sine Fourier series).

    u(eta, t) = F eta (H - eta) / (2 nu)
                - sum_{k odd} 4 F H^2 / (nu k^3 pi^3) sin(k pi eta / H) exp(-nu k^2 pi^2 t / H^2)
    """
    u = F * eta * (H - eta) / (2.0 * nu)
    for kk in range(1, 2 * terms, 2):
        u = u - 4.0 * F * H * H / (nu * kk**3 * np.pi**3) * np.sin(kk * np.pi * eta / H) * \
            np.exp(-nu * kk * kk * np.pi * np.pi * t / (H * H))
    return u


def smagorinsky_poiseuille(eta: np.ndarray, H: float, F: float, nu0: float, c_smag: float,
                           rho0: float = 1.0) -> np.ndarray:
    """Steady plane channel flow between walls at eta = 0 and H under a uniform body force F
    along the walls, with the Smagorinsky viscosity nu = nu0 + C_s^2 |S|, |S| = sqrt(2 S:S).

    For a velocity u(eta) along the walls the strain has one independent component,
    S_{eta u} = u'/2, so 2 S:S = 4 (u'/2)^2 = u'^2 and |S| = |u'|. The stress balance at
    distance s = |eta - H/2| from the mid-plane, rho0 (nu0 + C_s^2 |u'|) |u'| = F s, is a
    quadratic in |u'| with the positive root
      |u'|(s) = (q(s) - nu0) / (2 C_s^2),   q(s) = sqrt(nu0^2 + 4 C_s^2 F s / rho0).
    With u = 0 at the wall (s = H/2) and the substitution s = (q^2 - nu0^2) rho0 / (4 C_s^2 F),
      u = int_s^{H/2} |u'| ds'
        = (H/2 - s) / (2 (q_w + q)) [ nu0 (e_w + e) + (2/3) C_s^2 (e_w^2 + e_w e + e^2) ],
    where q_w = q(H/2) and e(s) = (q(s) - nu0) / C_s^2 = 4 F s / (rho0 (q(s) + nu0)); this
    form has no cancellation as C_s -> 0, where it tends to the Newtonian profile
    F ((H/2)^2 - s^2) / (2 rho0 nu0).
    """
    c2 = c_smag * c_smag
    half = H / 2.0
    s = np.abs(np.asarray(eta, dtype=np.float64) - half)

    def q(dist):
        return np.sqrt(nu0 * nu0 + 4.0 * c2 * F * dist / rho0)

    def e(dist, qd):
        return 4.0 * F * dist / (rho0 * (qd + nu0))

    qw, qs = q(half), q(s)
    ew, es = e(half, qw), e(s, qs)
    return (half - s) / (2.0 * (qw + qs)) * (nu0 * (ew + es) + (2.0 / 3.0) * c2 * (ew * ew + ew * es + es * es))
