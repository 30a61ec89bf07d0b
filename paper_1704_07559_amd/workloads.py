"""The benchmarked workloads C0-C4 as data.

Each JSON file under ``configs/`` records, for one workload, every constant the paper leaves
open (the relaxation rates of the non-viscous moments, the molecular viscosity, the
Smagorinsky constant, the power-law constants and clamps, the force, the initial field and
its seed, the run length) together with the readings that fix them. ``params`` turns a
workload into library parameters; nothing here computes any part of the method.

    from paper_1704_07559_amd import workloads
    cfg = workloads.load("C1")
    p = workloads.params(cfg)            # capi.Params of the 256^3 LES
"""
from __future__ import annotations

import json
from pathlib import Path

from . import capi

CONFIG_DIR = Path(__file__).resolve().parent / "configs"
FILES = {"C0": "c0_tgv32", "C1": "c1_les256", "C2": "c2_channel", "C3": "c3_les384_half", "C4": "c4_adjoint128"}


def load(name: str) -> dict:
    """A workload by its label (C0..C4) or file stem."""
    stem = FILES.get(name, name)
    with open(CONFIG_DIR / f"{stem}.json") as f:
        return json.load(f)


def nu_of_tau(tau_nu: float) -> float:
    """Lattice viscosity of the relaxation time tau_nu: nu = (tau_nu - 1/2) / 3."""
    return (tau_nu - 0.5) / 3.0


def rates_d3q19(tau_nu: float) -> list:
    """D3Q19 rates (reading R3): s_e = 1.19, s_eps = s_pi = 1.4, s_q = 1.2, s_t = 1.98, the
    conserved rows 0, s_nu = 1/tau_nu in slots 9, 11, 13, 14, 15."""
    sn = 1.0 / tau_nu
    return [0.0, 1.19, 1.4, 0.0, 1.2, 0.0, 1.2, 0.0, 1.2, sn, 1.4, sn, 1.4, sn, sn, sn, 1.98, 1.98, 1.98]


def rates_d3q15(tau_nu: float) -> list:
    """D3Q15 rates (rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, p_ww, p_xy, p_yz, p_xz,
    m_xyz; reading R16): s_e = 1.6, s_eps = 1.2, s_q = 1.6, s_m = 1.2, s_nu = 1/tau_nu."""
    sn = 1.0 / tau_nu
    return [0.0, 1.6, 1.2, 0.0, 1.6, 0.0, 1.6, 0.0, 1.6, sn, sn, sn, sn, sn, 1.2]


def rates_d2q9(tau_nu: float) -> list:
    """D2Q9 rates (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy; reading R12)."""
    sn = 1.0 / tau_nu
    return [0.0, 1.19, 1.4, 0.0, 1.2, 0.0, 1.2, sn, sn]


_LATTICE = {"D3Q19": (capi.LBM_D3Q19, rates_d3q19), "D3Q15": (capi.LBM_D3Q15, rates_d3q15),
            "D2Q9": (capi.LBM_D2Q9, rates_d2q9)}
_STORAGE = {"f32": capi.LBM_F32, "f16": capi.LBM_F16, "bf16": capi.LBM_BF16}
_DRIVE = {"yu": capi.LBM_STRAIN_YU, "chai": capi.LBM_STRAIN_CHAI}


def params(cfg: dict, storage: str | None = None, n_pl: float | None = None, lattice: str | None = None,
           grid: dict | None = None) -> capi.Params:
    """Library parameters of a workload. ``storage`` picks one of the workload's storage types
    (default: its first), ``n_pl`` one of a power-law workload's indices (default: its first),
    ``lattice`` and ``grid`` override the workload's (the same LES on another lattice or box).
    A random force field is not part of the parameters: the caller generates it from the
    recipe in cfg["force"] and sets ``force_field``."""
    lat = lattice or cfg["lattice"]
    lat_id, rates = _LATTICE[lat]
    g = grid or cfg["grid"]
    st = storage or cfg["storage"][0]
    if st not in cfg["storage"] and grid is None and lattice is None:
        raise ValueError(f"workload {cfg['name']} has no {st} storage")
    s = rates(cfg["tau_nu"])
    p = capi.Params(nx=g["nx"], ny=g["ny"], nz=g["nz"], lattice=lat_id, storage=_STORAGE[st], rho0=cfg["rho0"],
                    s=list(s) + [0.0] * (19 - len(s)), walls_y=int(cfg["walls_y"]))
    if lat == "D3Q19":
        p.omega_eps, p.omega_epsj, p.omega_xx = cfg["omegas"]
    v = cfg["viscosity"]
    if v["kind"] == "smagorinsky":
        p.visc_kind, p.visc_strain, p.c_smag = capi.LBM_VISC_SMAGORINSKY, _DRIVE[v["drive"]], v["c_smag"]
        p.nu0 = nu_of_tau(cfg["tau_nu"]) if v["nu0"] == "from tau_nu" else float(v["nu0"])
    elif v["kind"] == "powerlaw":
        n = v["n_pl"][0] if n_pl is None else n_pl
        if n not in v["n_pl"]:
            raise ValueError(f"workload {cfg['name']} has no power-law index {n}")
        F = cfg["force"]
        gamma_ref = (F[0] ** 2 + F[1] ** 2 + F[2] ** 2) ** 0.5 * g["ny"] / (2.0 * v["nu_ref"])
        p.visc_kind, p.visc_strain = capi.LBM_VISC_POWERLAW, _DRIVE[v["drive"]]
        p.K_pl, p.n_pl = v["nu_ref"] * gamma_ref ** (1.0 - n), n
        p.nu_min, p.nu_max = v["nu_min"], v["nu_max"]
    elif v["kind"] != "const":
        raise ValueError(f"unknown viscosity kind {v['kind']}")
    F = cfg["force"]
    if isinstance(F, list):
        p.force = tuple(float(a) for a in F)
    return p
