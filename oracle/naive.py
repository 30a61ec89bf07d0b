"""Per-node loop form of the D3Q19 step, for brute-force checks on tiny grids.

TEST INFRASTRUCTURE ONLY. Each node is visited in a Python loop; neighbours are found by
explicit modular index arithmetic (a pull: node x receives population i from x - c_i)
instead of ``np.roll``, and every per-node quantity is a 19-vector. It exists to pin the
vectorised oracle (``d3q19``): array axes, roll directions, broadcasting of per-node rates
and the bounce-back rule are all re-derived here independently. Only the paper's tables
and formulas are shared with ``d3q19`` (imported from it), not its array code.
"""
from __future__ import annotations

import numpy as np

from . import d3q19 as d


def _rates(p: d.Params, s_nu: float) -> np.ndarray:
    s = p.s.copy()
    for k in d.NU_SLOTS:
        s[k] = s_nu
    return s


def _node_strain_yu(mneq, s1, s9, r0):
    return [
        -(s1 * mneq[1] + 19 * s9 * mneq[9]) / (38 * r0),
        -(2 * s1 * mneq[1] - 19 * s9 * (mneq[9] - 3 * mneq[11])) / (76 * r0),
        -(2 * s1 * mneq[1] - 19 * s9 * (mneq[9] + 3 * mneq[11])) / (76 * r0),
        -3 * s9 * mneq[13] / (2 * r0),
        -3 * s9 * mneq[14] / (2 * r0),
        -3 * s9 * mneq[15] / (2 * r0),
    ]


def step(g: np.ndarray, p: d.Params, s_nu_field: np.ndarray):
    """One collide + stream of the pre-collision state g (19, nz, ny, nx), node by node.

    Returns (g_next, S_yu, S_chai, s_nu_new) with the strains of the incoming state.
    """
    _, nz, ny, nx = g.shape
    F = p.force_field((nz, ny, nx))
    post = np.empty_like(g)
    S_yu = np.empty((6, nz, ny, nx))
    S_chai = np.empty((6, nz, ny, nx))
    s_new = np.empty((nz, ny, nx))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                gi = g[:, z, y, x].copy()
                Fx = F[:, z, y, x]
                drho = gi.sum()
                j = np.array([sum(d.C[a, i] * gi[i] for i in range(19)) for a in range(3)]) + 0.5 * Fx
                m = d.T @ gi
                meq = d.m_eq(np.array(drho), j, p.rho0, p.omega_eps, p.omega_epsj, p.omega_xx)
                sp = _rates(p, s_nu_field[z, y, x])
                Sy = _node_strain_yu(m - meq, sp[1], sp[9], p.rho0)
                # Chai: build the 19x19 matrix T^-1 diag(s) T explicitly at this node.
                A = d.TINV @ np.diag(sp) @ d.T
                fneq = gi - d.g_eq(np.array(drho), j, p.rho0)
                Af = A @ fneq
                Sc = []
                for a, b in ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)):
                    N = sum(d.C[a, i] * d.C[b, i] * Af[i] for i in range(19))
                    Sc.append(-N / (2 * p.rho0 * d.CS2))
                S_yu[:, z, y, x] = Sy
                S_chai[:, z, y, x] = Sc
                drive = np.array(Sy if p.visc_strain == "yu" else Sc).reshape(6, 1, 1, 1)
                sn = float(d.viscosity_rate(drive, p, float(p.s[9])).ravel()[0])
                s_new[z, y, x] = sn
                s = _rates(p, sn)
                Fbar = d.guo_force_populations(j, Fx, p.rho0)
                mpost = m - s * (m - meq) + (1 - s / 2) * (d.T @ Fbar)
                post[:, z, y, x] = d.TINV @ mpost
    out = np.empty_like(g)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                for i in range(19):
                    cx, cy, cz = (int(v) for v in d.C[:, i])
                    ys = y - cy
                    if p.walls_y and not (0 <= ys < ny):
                        out[i, z, y, x] = post[d.OPP[i], z, y, x]
                    else:
                        out[i, z, y, x] = post[i, (z - cz) % nz, ys % ny, (x - cx) % nx]
    return out, S_yu, S_chai, s_new
