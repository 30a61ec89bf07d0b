"""Per-node loop form of the D2Q9 and D3Q15 steps, for brute-force checks on tiny grids.

TEST INFRASTRUCTURE ONLY. The counterpart of ``naive`` for the other two lattices: each node
is visited in a Python loop, neighbours come from explicit modular index arithmetic (node x
receives population i from x - c_i, or opp(i) of itself across a y-wall), the Chai strain
is the explicit per-node matrix T^-1 diag(s) T contracted with c c, and the Yu-type strain is
the closed form the Section 5.4 route gives for each lattice, written out here:
  D2Q9 : S_xx, S_yy = -(s_e m1 +- 3 s_nu m7) / (4 rho0),  S_xy = -3 s_nu m8 / (2 rho0)
  D3Q15: S_xx = -(s_e m1 + s_nu m9) / (2 rho0),
         S_yy, S_zz = -(2 s_e m1 - s_nu m9 +- 3 s_nu m10) / (4 rho0),
         S_xy, S_yz, S_xz = -3 s_nu m11, m12, m13 / (2 rho0).
Only the lattice tables and equilibria are taken from ``d2q9`` / ``d3q15``, not their array
code (rolls, broadcasting, the numeric Section 5.4 route).
"""
from __future__ import annotations

import numpy as np


def _yu_closed_form(q, m, se, sn, r0):
    if q == 9:
        return [-(se * m[1] + 3 * sn * m[7]) / (4 * r0), -(se * m[1] - 3 * sn * m[7]) / (4 * r0),
                -3 * sn * m[8] / (2 * r0)]
    return [-(se * m[1] + sn * m[9]) / (2 * r0),
            -(2 * se * m[1] - sn * m[9] + 3 * sn * m[10]) / (4 * r0),
            -(2 * se * m[1] - sn * m[9] - 3 * sn * m[10]) / (4 * r0),
            -3 * sn * m[11] / (2 * r0), -3 * sn * m[12] / (2 * r0), -3 * sn * m[13] / (2 * r0)]


def step(mod, g: np.ndarray, p, s_nu_field: np.ndarray):
    """One collide + stream of g (Q, nz, ny, nx) on the lattice of ``mod`` (d2q9 or d3q15),
    node by node, lagged or constant viscosity. Returns (g_next, S_yu, S_chai, s_nu_new)."""
    Q, nz, ny, nx = g.shape
    dim = mod.C.shape[0]
    pairs = ((0, 0), (1, 1), (0, 1)) if dim == 2 else ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2))
    F = p.force_field((nz, ny, nx))
    post = np.empty_like(g)
    nc = len(pairs)
    S_yu = np.empty((nc, nz, ny, nx))
    S_chai = np.empty((nc, nz, ny, nx))
    s_new = np.empty((nz, ny, nx))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                gi = g[:, z, y, x].copy()
                Fx = F[:, z, y, x]
                drho = gi.sum()
                j = np.array([sum(mod.C[a, i] * gi[i] for i in range(Q)) for a in range(dim)]) + 0.5 * Fx
                m = mod.T @ gi
                meq = mod.m_eq(np.array(drho), j, p.rho0)
                sp = p.s.copy()
                for k in mod.NU_SLOTS:
                    sp[k] = s_nu_field[z, y, x]
                Sy = _yu_closed_form(Q, m - meq, sp[1], sp[mod.NU_SLOTS[0]], p.rho0)
                A = mod.TINV @ np.diag(sp) @ mod.T
                Af = A @ (gi - mod.g_eq(np.array(drho), j, p.rho0))
                Sc = [-sum(mod.C[a, i] * mod.C[b, i] * Af[i] for i in range(Q)) / (2 * p.rho0 * mod.CS2)
                      for a, b in pairs]
                S_yu[:, z, y, x] = Sy
                S_chai[:, z, y, x] = Sc
                drive = np.array(Sy if p.visc_strain == "yu" else Sc).reshape((nc,) + (1,) * 3)
                sn = float(np.asarray(mod.viscosity_rate(drive, p, float(p.s[mod.NU_SLOTS[0]]))).ravel()[0])
                s_new[z, y, x] = sn
                s = p.s.copy()
                for k in mod.NU_SLOTS:
                    s[k] = sn
                Fbar = mod.guo_force_populations(j, Fx, p.rho0)
                post[:, z, y, x] = mod.TINV @ (m - s * (m - meq) + (1 - s / 2) * (mod.T @ Fbar))
    out = np.empty_like(g)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                for i in range(Q):
                    c = [int(v) for v in mod.C[:, i]] + [0] * (3 - dim)
                    ys = y - c[1]
                    if p.walls_y and not (0 <= ys < ny):
                        out[i, z, y, x] = post[mod.OPP[i], z, y, x]
                    else:
                        out[i, z, y, x] = post[i, (z - c[2]) % nz, ys % ny, (x - c[0]) % nx]
    return out, S_yu, S_chai, s_new
