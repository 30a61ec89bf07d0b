"""FP64 oracle: discrete adjoint of the D3Q19 MRT step and of a strain-squared loss.

TEST INFRASTRUCTURE ONLY. The paper has no adjoint; this is the exact transpose of the
oracle's own forward step (``d3q19.collide`` + ``d3q19.stream``) for a constant viscosity,
used to check the hand-written adjoint kernel (strain-dependent viscosities:
``adjoint_visc``).

Forward problem (all FP64):
  g^0      = g^eq(0, rho0 u0)                         (delta-rho form of Eq. edf)
  g^{n+1}  = P C(g^n, F),  n = 0..N-1                 (Eq. mrteq; C collision, P streaming)
  J        = sum_x S(g^N, F) : S(g^N, F)               (Yu strain, Eq. LuoS; off-diagonal
                                                        components counted twice)
with a body-force field F entering through j = sum c g + F/2 and the Guo term.

Jacobians. The collision is a polynomial of degree two in (g, F) for a constant viscosity:
m^eq is quadratic in j, the Guo term is bilinear in (j, F). Its derivatives are therefore
obtained from the pinned forward functions by central differences, which are exact for
polynomials of degree <= 2 at any step size (here a unit step); no derivative is written
out by hand a second time.
"""
from __future__ import annotations

import numpy as np

from . import d3q19 as d

Q = d.Q


# ---------------------------------------------------------------------------------------
# Exact derivatives of the quadratic building blocks
# ---------------------------------------------------------------------------------------

def dmeq_ddrho(p: d.Params) -> np.ndarray:
    """d m^eq / d delta_rho (m^eq is linear in delta_rho): shape (19,)."""
    z = np.zeros(3)
    return (d.m_eq(np.array(1.0), z, p.rho0, p.omega_eps, p.omega_epsj, p.omega_xx)
            - d.m_eq(np.array(-1.0), z, p.rho0, p.omega_eps, p.omega_epsj, p.omega_xx)) / 2.0


def dmeq_dj(j: np.ndarray, p: d.Params) -> np.ndarray:
    """d m^eq / d j at j (quadratic in j): j (3, M) -> (19, 3, M)."""
    M = j.shape[1]
    out = np.empty((Q, 3, M))
    z = np.zeros(M)
    for k in range(3):
        e = np.zeros((3, 1))
        e[k] = 1.0
        out[:, k] = (d.m_eq(z, j + e, p.rho0, p.omega_eps, p.omega_epsj, p.omega_xx)
                     - d.m_eq(z, j - e, p.rho0, p.omega_eps, p.omega_epsj, p.omega_xx)) / 2.0
    return out


def dFbar_dj(j: np.ndarray, F: np.ndarray, p: d.Params) -> np.ndarray:
    """d F-bar / d j (F-bar linear in j): (19, 3, M)."""
    M = j.shape[1]
    out = np.empty((Q, 3, M))
    for k in range(3):
        e = np.zeros((3, 1))
        e[k] = 1.0
        out[:, k] = (d.guo_force_populations(j + e, F, p.rho0) - d.guo_force_populations(j - e, F, p.rho0)) / 2.0
    return out


def dFbar_dF(j: np.ndarray, F: np.ndarray, p: d.Params) -> np.ndarray:
    """d F-bar / d F (F-bar linear in F): (19, 3, M)."""
    M = j.shape[1]
    out = np.empty((Q, 3, M))
    for k in range(3):
        e = np.zeros((3, 1))
        e[k] = 1.0
        out[:, k] = (d.guo_force_populations(j, F + e, p.rho0) - d.guo_force_populations(j, F - e, p.rho0)) / 2.0
    return out


def half_source_jacobians(j: np.ndarray, F: np.ndarray, p: d.Params):
    """d h / d j and d h / d F, each (19, 3, M), of the half Guo source h = T F-bar / 2 that the
    force-corrected strain adds to the non-equilibrium moments (both zero without the
    correction): the strain input is X = T g - m^eq(delta_rho, j) + h(j, F)."""
    M = j.shape[1]
    if not p.force_corrected:
        z = np.zeros((Q, 3, M))
        return z, z
    return (0.5 * np.einsum("ri,ikm->rkm", d.T, dFbar_dj(j, F, p)),
            0.5 * np.einsum("ri,ikm->rkm", d.T, dFbar_dF(j, F, p)))


def yu_map(p: d.Params, s_nu: float) -> np.ndarray:
    """The 6x19 linear map m^neq -> S of Eq. LuoS (columns = strain_yu of unit vectors)."""
    Y = np.empty((6, Q))
    for k in range(Q):
        e = np.zeros(Q)
        e[k] = 1.0
        Y[:, k] = d.strain_yu(e, float(p.s[1]), s_nu, p.rho0)
    return Y


# ---------------------------------------------------------------------------------------
# Per-node Jacobians of the collision (Eq. mrteqvT with the Guo term)
# ---------------------------------------------------------------------------------------

def collision_jacobians(g: np.ndarray, F: np.ndarray, p: d.Params, rates: np.ndarray | None = None):
    """Per-node dg*/dg (M, 19, 19) and dg*/dF (M, 19, 3) of the collision at state g, with
    the relaxation rates held fixed.

    With m = T g, delta_rho = sum g, j = C g + F/2 and
      m* = m - L (m - m^eq(delta_rho, j)) + (I - L/2) T F-bar(j, F),  g* = T^-1 m*,
      dm*/dg = (I - L) T + L dm^eq/dg + (I - L/2) T dF-bar/dj C
      dm*/dF = L dm^eq/dj / 2 + (I - L/2) T (dF-bar/dF + dF-bar/dj / 2)
    with L = diag(s): the rates of p (constant viscosity), or ``rates`` (19, M) per node;
    diagonal products are written as broadcasts. (The strain, force-corrected or not, does
    not enter the collision at fixed rates.)
    """
    if rates is None and p.visc_kind != "const":
        raise ValueError("a strain-dependent viscosity needs the per-node rates")
    q, *shape = g.shape
    M = int(np.prod(shape))
    gf = g.reshape(Q, M)
    Ff = F.reshape(3, M)
    j = d.C.astype(float) @ gf + 0.5 * Ff
    Cf = d.C.astype(float)
    dmr = dmeq_ddrho(p)                       # (19,)
    dmj = dmeq_dj(j, p)                       # (19, 3, M)
    dfj = dFbar_dj(j, Ff, p)                  # (19, 3, M)
    dfF = dFbar_dF(j, Ff, p)                  # (19, 3, M)
    # dm^eq/dg = dm^eq/d(drho) 1^T + dm^eq/dj C            -> (M, 19, 19)
    dmeq_dg = dmr[None, :, None] * np.ones((1, 1, Q)) + np.einsum("rkm,ki->mri", dmj, Cf, optimize=True)
    TdfjC = np.einsum("ri,ikm,kl->mrl", d.T, dfj, Cf, optimize=True)      # T dF-bar/dj C
    sv = p.s[None, :, None] if rates is None else rates.T[:, :, None]     # L = diag(s)
    dmstar_dg = (1.0 - sv) * d.T[None] + sv * dmeq_dg + (1.0 - sv / 2.0) * TdfjC
    Jgg = np.matmul(d.TINV[None], dmstar_dg)
    TdfF = np.einsum("ri,ikm->mrk", d.T, dfF + dfj / 2.0, optimize=True)
    dmstar_dF = sv * np.transpose(dmj, (2, 0, 1)) / 2.0 + (1.0 - sv / 2.0) * TdfF
    JgF = np.matmul(d.TINV[None], dmstar_dF)
    return Jgg, JgF


# ---------------------------------------------------------------------------------------
# Transpose of the streaming map
# ---------------------------------------------------------------------------------------

def stream_transpose(lam: np.ndarray, walls_y: bool = False) -> np.ndarray:
    """P^T of ``d3q19.stream``: lam_tilde_i(y) = lam_i(y + c_i), or lam_opp(i)(y) when
    y + c_i lies beyond a y-wall (the transpose of halfway bounce-back)."""
    out = np.empty_like(lam)
    ny = lam.shape[2]
    for i in range(Q):
        cx, cy, cz = (int(v) for v in d.C[:, i])
        out[i] = np.roll(lam[i], shift=(-cz, -cy, -cx), axis=(0, 1, 2))
    if walls_y:
        for i in range(Q):
            cy = int(d.C[1, i])
            if cy == 1:      # y + c_y leaves through the upper wall at y = ny-1
                out[i][:, ny - 1, :] = lam[d.OPP[i]][:, ny - 1, :]
            elif cy == -1:   # ... through the lower wall at y = 0
                out[i][:, 0, :] = lam[d.OPP[i]][:, 0, :]
    return out


def adjoint_step(lam_next: np.ndarray, g: np.ndarray, F: np.ndarray, p: d.Params):
    """One reverse step: given lam^{n+1} = dJ/dg^{n+1} and the forward state g^n, return
    (lam^n, dJ/dF contribution of this step)."""
    lt = stream_transpose(lam_next, p.walls_y)
    Jgg, JgF = collision_jacobians(g, F, p)
    M = Jgg.shape[0]
    lf = lt.reshape(Q, M)
    lam = np.matmul(lf.T[:, None, :], Jgg)[:, 0, :].T.reshape(g.shape)            # Jgg^T lam
    gF = np.matmul(lf.T[:, None, :], JgF)[:, 0, :].T.reshape((3,) + g.shape[1:])  # JgF^T lam
    return lam, gF


# ---------------------------------------------------------------------------------------
# The loss and its seed
# ---------------------------------------------------------------------------------------

def strain_loss(g: np.ndarray, F: np.ndarray, p: d.Params) -> float:
    """J = sum_x S:S of the Yu strain of g (rates of p: constant viscosity)."""
    S = d.strain_of_state(g, _with_force(p, F), np.full(g.shape[1:], float(p.s[9])), "yu")
    return float(d.strain_sq(S).sum())


def _with_force(p: d.Params, F: np.ndarray) -> d.Params:
    q = d.Params(**{k: getattr(p, k) for k in p.__dataclass_fields__})
    q.force = F
    return q


def strain_loss_seed(g: np.ndarray, F: np.ndarray, p: d.Params):
    """(J, dJ/dg, dJ/dF) for J = sum_x S:S with S = Y X, X = T g - m^eq(delta_rho, j) + h(j, F)
    (h the half Guo source of the force-corrected strain, else 0), j = C g + F/2:
      dJ/dg = (T - dm^eq/dg + dh/dj C)^T sigma,
      dJ/dF = (-dm^eq/dj / 2 + dh/dj / 2 + dh/dF)^T sigma,   sigma = Y^T (2 W S),
    W = diag(1, 1, 1, 2, 2, 2)."""
    q, *shape = g.shape
    M = int(np.prod(shape))
    gf = g.reshape(Q, M)
    Ff = F.reshape(3, M)
    drho = gf.sum(axis=0)
    j = d.C.astype(float) @ gf + 0.5 * Ff
    m = d.T @ gf
    meq = d.m_eq(drho, j, p.rho0, p.omega_eps, p.omega_epsj, p.omega_xx)
    dhj, dhF = half_source_jacobians(j, Ff, p)
    X = m - meq
    if p.force_corrected:
        X = X + 0.5 * (d.T @ d.guo_force_populations(j, Ff, p.rho0))
    Y = yu_map(p, float(p.s[9]))
    S = Y @ X
    W = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])
    J = float((W[:, None] * S * S).sum())
    sigma = Y.T @ (2.0 * W[:, None] * S)                       # (19, M) in moment space
    dmr = dmeq_ddrho(p)
    dmj = dmeq_dj(j, p)
    Cf = d.C.astype(float)
    bj = np.einsum("rkm,rm->km", dmj, sigma)                   # (dm^eq/dj)^T sigma
    hj = np.einsum("rkm,rm->km", dhj, sigma)                   # (dh/dj)^T sigma
    hF = np.einsum("rkm,rm->km", dhF, sigma)                   # (dh/dF)^T sigma
    lam = d.T.T @ sigma - np.ones((Q, 1)) * (dmr @ sigma)[None] + Cf.T @ (hj - bj)
    gF = 0.5 * (hj - bj) + hF
    return J, lam.reshape(g.shape), gF.reshape((3,) + tuple(shape))


def init_adjoint(lam0: np.ndarray, u0: np.ndarray, p: d.Params) -> np.ndarray:
    """grad_u0 = sum_i lam0_i d g^eq_i(0, rho0 u0) / d u0 (g^eq quadratic in u0: exact
    central differences)."""
    shape = u0.shape[1:]
    out = np.empty((3,) + shape)
    z = np.zeros(shape)
    for k in range(3):
        e = np.zeros((3,) + (1,) * len(shape))
        e[k] = 1.0
        dg = (d.g_eq(z, p.rho0 * (u0 + e), p.rho0) - d.g_eq(z, p.rho0 * (u0 - e), p.rho0)) / 2.0
        out[k] = (lam0 * dg).sum(axis=0)
    return out


# ---------------------------------------------------------------------------------------
# Whole problem: forward loss, gradient with checkpointing
# ---------------------------------------------------------------------------------------

def forward(u0: np.ndarray, F: np.ndarray, p: d.Params, nsteps: int) -> float:
    """J after nsteps; with a strain-dependent viscosity the strain of the final state takes
    the rate the model gives it (the lagged field, or the implicitly solved rate)."""
    pf = _with_force(p, F)
    sim = d.Simulation(pf, d.init_populations(np.zeros(u0.shape[1:]), u0, pf))
    sim.step(nsteps)
    if p.visc_kind == "const":
        return strain_loss(sim.g, F, p)
    return float(d.strain_sq(sim.strain("yu")).sum())


def gradient(u0: np.ndarray, F: np.ndarray, p: d.Params, nsteps: int, every: int | None = None):
    """(J, dJ/du0, dJ/dF) by the discrete adjoint. States are checkpointed every ``every``
    steps in the forward sweep and recomputed segment by segment in the reverse sweep."""
    if p.visc_kind != "const":
        from .adjoint_visc import gradient_visc
        return gradient_visc(u0, F, p, nsteps, every)
    every = every or nsteps
    pf = _with_force(p, F)
    sim = d.Simulation(pf, d.init_populations(np.zeros(u0.shape[1:]), u0, pf))
    checkpoints = {}
    for n in range(nsteps):
        if n % every == 0:
            checkpoints[n] = sim.g.copy()
        sim.step(1)
    J, lam, gF = strain_loss_seed(sim.g, F, p)
    for start in sorted(checkpoints, reverse=True):
        stop = min(start + every, nsteps)
        seg = d.Simulation(pf, checkpoints[start])
        states = []
        for _ in range(start, stop):
            states.append(seg.g.copy())
            seg.step(1)
        for g in reversed(states):
            lam, dF = adjoint_step(lam, g, F, pf)
            gF = gF + dF
    return J, init_adjoint(lam, u0, p), gF
