"""FP64 oracle: discrete adjoint of the D3Q19 step with a strain-dependent viscosity.

TEST INFRASTRUCTURE ONLY. The paper has no adjoint. This extends the constant-viscosity
adjoint of ``adjoint`` to the viscosity models of the forward oracle:
  lagged Smagorinsky / power law : the state is (g, s_nu field); the strain of step n uses
                                   the field s_prev, the collision relaxes with
                                   s_new = h(gamma), h(gamma) = 1 / (3 nu(gamma) + 1/2),
                                   and s_new becomes the field of step n+1;
  implicit Smagorinsky           : the state is g; s_new solves
                                   G(s) = s (3 nu(gamma(S(s))) + 1/2) - 1 = 0.
gamma = |S| = sqrt(2 S:S). Eq. LuoS is affine in s_nu, so per node
  S(s) = (Y_e + s Y_n) m^neq,   m^neq = T g - m^eq(delta_rho, j),  j = C g + F/2,
with Y_e the s_e part and Y_n the s_nu part at unit rate (the Chai strain is the same
function, Section 5.1, so the derivative is taken on this form for either drive). With the
force-corrected strain, m^neq in S is replaced by X = m^neq + h, h = T F-bar / 2 the half
Guo source, a bilinear function of (j, F) whose derivatives join the chain rule.

The collision m* = m - L(s_new)(m - m^eq) + (I - L/2) T F-bar depends on (g, F) with the
rates held fixed (``adjoint.collision_jacobians`` at the node's rates) and through s_new:
  dm*_k/ds_new = -(m^neq_k + (T F-bar)_k / 2) on the s_nu rows k = 9, 11, 13, 14, 15,
a rank-one term per node. The rate's own derivatives follow by the chain rule:
  lagged   : ds_new/dm^neq = h'(gamma) (dgamma/dS)^T (Y_e + s_prev Y_n),
             ds_new/ds_prev = h'(gamma) (dgamma/dS) . (Y_n m^neq),  h' = -3 nu'(gamma) h^2
  implicit : ds/dm^neq = -(dG/dm^neq) / (dG/ds)  (implicit function theorem)
with dgamma/dS = 2 W S / gamma, W = (1, 1, 1, 2, 2, 2). Each piece is checked against
central differences of the forward oracle in the tests.
"""
from __future__ import annotations

import numpy as np

from . import adjoint as adj
from . import d3q19 as d

Q = d.Q
W6 = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])


def strain_maps(p: d.Params):
    """(Y_e, Y_n), each 6x19: S = (Y_e + s_nu Y_n) m^neq (Eq. LuoS)."""
    Ye = np.empty((6, Q))
    Yn = np.empty((6, Q))
    for k in range(Q):
        e = np.zeros(Q)
        e[k] = 1.0
        Ye[:, k] = d.strain_yu(e, float(p.s[1]), 0.0, p.rho0)
        Yn[:, k] = d.strain_yu(e, 0.0, 1.0, p.rho0)
    return Ye, Yn


def nu_slope(gamma: np.ndarray, p: d.Params) -> np.ndarray:
    """d nu / d gamma of the lagged models: C_s^2 (Smagorinsky); (n-1) nu / gamma where the
    power law is not clamped and gamma > 0, else 0."""
    if p.visc_kind == "smagorinsky":
        return np.full(gamma.shape, p.c_smag**2)
    if p.visc_kind == "powerlaw":
        out = np.zeros_like(gamma)
        pos = gamma > 0.0
        nu = np.zeros_like(gamma)
        nu[pos] = p.K_pl * np.power(gamma[pos], p.n_pl - 1.0)
        free = pos & (nu > p.nu_min) & (nu < p.nu_max)
        out[free] = (p.n_pl - 1.0) * nu[free] / gamma[free]
        return out
    raise ValueError(p.visc_kind)


def local_moments(g: np.ndarray, F: np.ndarray, p: d.Params):
    """Flattened per-node quantities of the collision: (j (3, M), m^neq (19, M), T F-bar)."""
    M = g[0].size
    gf = g.reshape(Q, M)
    Ff = F.reshape(3, M)
    drho = gf.sum(axis=0)
    j = d.C.astype(float) @ gf + 0.5 * Ff
    mneq = d.T @ gf - d.m_eq(drho, j, p.rho0, p.omega_eps, p.omega_epsj, p.omega_xx)
    SF = d.T @ d.guo_force_populations(j, Ff, p.rho0)
    return j, mneq, SF


def _dgamma_dS(S: np.ndarray):
    gamma = d.strain_norm(S)
    safe = np.where(gamma > 0.0, gamma, 1.0)
    return gamma, np.where(gamma > 0.0, 2.0 * W6[:, None] * S / safe, 0.0)


def rate_sensitivities(mneq: np.ndarray, s_prev: np.ndarray | None, p: d.Params):
    """(s_new (M,), ds_new/dm^neq (M, 19), ds_new/ds_prev (M,)) per node."""
    Ye, Yn = strain_maps(p)
    Pm, Am = Ye @ mneq, Yn @ mneq
    M = mneq.shape[1]
    if p.visc_kind == "smagorinsky_implicit":
        s = d.implicit_smagorinsky_rate(lambda sv: Pm + sv * Am, p, (M,))
        gamma, dgdS = _dgamma_dS(Pm + s * Am)
        c, k = 3.0 * p.nu0 + 0.5, 3.0 * p.c_smag**2
        dG_ds = c + k * gamma + s * k * (dgdS * Am).sum(axis=0)
        dG_dm = (s * k)[:, None] * (dgdS.T @ Ye + s[:, None] * (dgdS.T @ Yn))
        return s, -dG_dm / dG_ds[:, None], np.zeros(M)
    S = Pm + s_prev * Am
    gamma, dgdS = _dgamma_dS(S)
    s = d.viscosity_rate(S, p, float(p.s[9]))
    dh = -3.0 * nu_slope(gamma, p) * s * s
    ds_dm = dh[:, None] * (dgdS.T @ Ye + s_prev[:, None] * (dgdS.T @ Yn))
    return s, ds_dm, dh * (dgdS * Am).sum(axis=0)


def strain_input(mneq: np.ndarray, SF: np.ndarray, p: d.Params) -> np.ndarray:
    """X, the moments the strain formulas take: m^neq, plus S_F / 2 for the force-corrected
    strain."""
    return mneq + 0.5 * SF if p.force_corrected else mneq


def _chain_X(dv_dX: np.ndarray, j: np.ndarray, F: np.ndarray, p: d.Params):
    """Per-node dv/dg (M, 19) and dv/dF (M, 3) of a quantity v with dv/dX (M, 19), through
    X = T g - m^eq(delta_rho, j) + h(j, F), j = C g + F/2."""
    Cf = d.C.astype(float)
    dmj = adj.dmeq_dj(j, p)                                                # (19, 3, M)
    dhj, dhF = adj.half_source_jacobians(j, F, p)
    dXj = dhj - dmj                                                        # dX/dj
    dX_dg = (d.T[None] - adj.dmeq_ddrho(p)[None, :, None] * np.ones((1, 1, Q))
             + np.einsum("rkm,ki->mri", dXj, Cf))
    dv_dg = np.einsum("mr,mri->mi", dv_dX, dX_dg)
    dv_dF = np.einsum("mr,rkm->mk", dv_dX, 0.5 * dXj + dhF)
    return dv_dg, dv_dF


def collision_jacobians_visc(g: np.ndarray, s_prev: np.ndarray | None, F: np.ndarray, p: d.Params) -> dict:
    """Per-node derivatives of (g, s_prev, F) -> (g*, s_new):
    Jgg (M, 19, 19), JgF (M, 19, 3), Jgs (19, M) = dg*/ds_prev, and the rate's own
    ds_dg (M, 19), ds_dF (M, 3), ds_dsp (M,)."""
    M = g[0].size
    j, mneq, SF = local_moments(g, F, p)
    sp = None if s_prev is None else s_prev.reshape(M)
    s, ds_dX, ds_dsp = rate_sensitivities(strain_input(mneq, SF, p), sp, p)
    Jgg, JgF = adj.collision_jacobians(g, F, p, rates=d.rates_field(p, s))
    ds_dg, ds_dF = _chain_X(ds_dX, j, F.reshape(3, M), p)
    e_nu = np.zeros((Q, 1))
    e_nu[list(d.NU_SLOTS)] = 1.0
    dg_ds = d.TINV @ (-(mneq + 0.5 * SF) * e_nu)                           # (19, M)
    return {
        "s": s,
        "Jgg": Jgg + np.einsum("im,ml->mil", dg_ds, ds_dg),
        "JgF": JgF + np.einsum("im,mk->mik", dg_ds, ds_dF),
        "Jgs": dg_ds * ds_dsp[None],
        "ds_dg": ds_dg,
        "ds_dF": ds_dF,
        "ds_dsp": ds_dsp,
    }


def adjoint_step_visc(lam_next: np.ndarray, lams_next: np.ndarray | None, g: np.ndarray,
                      s_prev: np.ndarray | None, F: np.ndarray, p: d.Params):
    """One reverse step. lam_next = dJ/dg^{n+1}; lams_next = dJ/d(s_nu field of step n+1)
    (lagged models; None for the implicit one). Returns (lam^n, lams^n, dJ/dF of this step)."""
    shape = g.shape[1:]
    M = g[0].size
    lt = adj.stream_transpose(lam_next, p.walls_y).reshape(Q, M)
    Jv = collision_jacobians_visc(g, s_prev, F, p)
    ls = np.zeros(M) if lams_next is None else lams_next.reshape(M)
    lam = np.einsum("mil,im->lm", Jv["Jgg"], lt) + Jv["ds_dg"].T * ls
    gF = np.einsum("mik,im->km", Jv["JgF"], lt) + Jv["ds_dF"].T * ls
    lams = None
    if lams_next is not None:
        lams = ((Jv["Jgs"] * lt).sum(axis=0) + Jv["ds_dsp"] * ls).reshape(shape)
    return lam.reshape(g.shape), lams, gF.reshape((3,) + shape)


def strain_loss_seed_visc(g: np.ndarray, s_prev: np.ndarray | None, F: np.ndarray, p: d.Params):
    """(J, dJ/dg, dJ/ds_prev or None, dJ/dF) for J = sum_x S:S of the final state, the strain
    taken at the model's rate (lagged field, or implicitly solved)."""
    shape = g.shape[1:]
    M = g[0].size
    j, mneq, SF = local_moments(g, F, p)
    X = strain_input(mneq, SF, p)
    Ye, Yn = strain_maps(p)
    Am = Yn @ X
    if p.visc_kind == "smagorinsky_implicit":
        s, ds_dm, _ = rate_sensitivities(X, None, p)
    else:
        s = s_prev.reshape(M)
    S = Ye @ X + s * Am
    J = float((W6[:, None] * S * S).sum())
    dJ_dS = 2.0 * W6[:, None] * S
    dJ_dm = Ye.T @ dJ_dS + s * (Yn.T @ dJ_dS)                              # (19, M)
    dJ_ds = (dJ_dS * Am).sum(axis=0)
    lams = None
    if p.visc_kind == "smagorinsky_implicit":
        dJ_dm = dJ_dm + ds_dm.T * dJ_ds
    else:
        lams = dJ_ds.reshape(shape)
    lam, gF = _chain_X(dJ_dm.T, j, F.reshape(3, M), p)
    return J, lam.T.reshape(g.shape), lams, gF.T.reshape((3,) + shape)


def gradient_visc(u0: np.ndarray, F: np.ndarray, p: d.Params, nsteps: int, every: int | None = None):
    """(J, dJ/du0, dJ/dF) by the discrete adjoint for a strain-dependent viscosity, with the
    states (g and, for the lagged models, the s_nu field) checkpointed every ``every`` steps."""
    every = every or nsteps
    lagged = p.visc_kind != "smagorinsky_implicit"
    pf = adj._with_force(p, F)
    sim = d.Simulation(pf, d.init_populations(np.zeros(u0.shape[1:]), u0, pf))
    checkpoints = {}
    for n in range(nsteps):
        if n % every == 0:
            checkpoints[n] = (sim.g.copy(), sim.s_nu.copy())
        sim.step(1)
    J, lam, lams, gF = strain_loss_seed_visc(sim.g, sim.s_nu if lagged else None, F, p)
    for start in sorted(checkpoints, reverse=True):
        stop = min(start + every, nsteps)
        seg = d.Simulation(pf, checkpoints[start][0])
        seg.s_nu = checkpoints[start][1].copy()
        states = []
        for _ in range(start, stop):
            states.append((seg.g.copy(), seg.s_nu.copy()))
            seg.step(1)
        for g, sp in reversed(states):
            lam, lams, dF = adjoint_step_visc(lam, lams, g, sp if lagged else None, F, pf)
            gF = gF + dF
    return J, adj.init_adjoint(lam, u0, p), gF
