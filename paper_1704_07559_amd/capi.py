"""ctypes binding of liblbm.so with the names of the C ABI (include/lbm.h).

Argument marshalling only: tensors become device pointers, the stream becomes a
hipStream_t handle, a non-zero lbm_status becomes an LBMError. Every computation runs in
the HIP kernels of the library. If the library is missing this module raises on import;
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from pathlib import Path
from typing import Optional, Sequence

_LIB_PATH = Path(os.environ.get("LBM_LIBRARY", Path(__file__).resolve().parent / "liblbm.so"))

if not _LIB_PATH.exists():
    raise ImportError(
        f"{_LIB_PATH} is missing: build the HIP library first "
        "(python -m paper_1704_07559_amd.build, or __graft_entry__.build())")

_lib = ctypes.CDLL(str(_LIB_PATH))

# enums (include/lbm.h)
LBM_OK, LBM_EINVAL, LBM_EHIP, LBM_ENOMEM, LBM_ESTATE, LBM_ENONFINITE, LBM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
LBM_D2Q9, LBM_D3Q15, LBM_D3Q19 = 9, 15, 19
LBM_F32, LBM_F16, LBM_BF16 = 0, 1, 2
LBM_STRAIN_NONE, LBM_STRAIN_YU, LBM_STRAIN_CHAI = 0, 1, 2
LBM_VISC_CONST, LBM_VISC_SMAGORINSKY, LBM_VISC_POWERLAW, LBM_VISC_SMAGORINSKY_IMPLICIT = 0, 1, 2, 3

EXPORTED = (
    "lbm_params_size", "lbm_population_bytes", "lbm_init", "lbm_step", "lbm_strain", "lbm_reduce", "lbm_get_populations",
    "lbm_set_populations", "lbm_state_bytes", "lbm_save_state", "lbm_load_state", "lbm_step_count",
    "lbm_set_step_count", "lbm_save_planes", "lbm_adjoint_planes", "lbm_adjoint_step", "lbm_adjoint_steps", "lbm_adjoint_steps_noalloc", "lbm_strain_loss_seed", "lbm_init_adjoint", "lbm_destroy",
    "lbm_status_string", "lbm_last_error", "lbm_stream_copy", "lbm_reduce_async",
)


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int), ("storage", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("walls_y", ctypes.c_int),
        ("rho0", ctypes.c_double),
        ("s", ctypes.c_double * 19),
        ("omega_eps", ctypes.c_double), ("omega_epsj", ctypes.c_double), ("omega_xx", ctypes.c_double),
        ("visc_kind", ctypes.c_int), ("visc_strain", ctypes.c_int),
        ("nu0", ctypes.c_double), ("c_smag", ctypes.c_double), ("K_pl", ctypes.c_double),
        ("n_pl", ctypes.c_double), ("nu_min", ctypes.c_double), ("nu_max", ctypes.c_double),
        ("force", ctypes.c_double * 3),
        ("force_field", ctypes.c_void_p),
        ("strain_force_correction", ctypes.c_int),
    ]


_vp = ctypes.c_void_p
_ctx_p = ctypes.c_void_p
_sig = {
    "lbm_params_size": (ctypes.c_size_t, []),
    "lbm_population_bytes": (ctypes.c_size_t, [ctypes.POINTER(lbm_params)]),
    "lbm_init": (ctypes.c_int, [ctypes.POINTER(_ctx_p), ctypes.POINTER(lbm_params), _vp, _vp, _vp, _vp, _vp, _vp]),
    "lbm_step": (ctypes.c_int, [_ctx_p, ctypes.c_int, _vp, ctypes.c_int, _vp, _vp]),
    "lbm_strain": (ctypes.c_int, [_ctx_p, ctypes.c_int, _vp, _vp]),
    "lbm_reduce": (ctypes.c_int, [_ctx_p, ctypes.POINTER(ctypes.c_double), _vp]),
    "lbm_reduce_async": (ctypes.c_int, [_ctx_p, _vp, _vp]),
    "lbm_get_populations": (ctypes.c_int, [_ctx_p, _vp, _vp]),
    "lbm_set_populations": (ctypes.c_int, [_ctx_p, _vp, _vp]),
    "lbm_state_bytes": (ctypes.c_size_t, [_ctx_p]),
    "lbm_save_state": (ctypes.c_int, [_ctx_p, _vp, _vp]),
    "lbm_load_state": (ctypes.c_int, [_ctx_p, _vp, _vp]),
    "lbm_step_count": (ctypes.c_longlong, [_ctx_p]),
    "lbm_set_step_count": (ctypes.c_int, [_ctx_p, ctypes.c_longlong]),
    "lbm_save_planes": (ctypes.c_int, [_ctx_p]),
    "lbm_adjoint_planes": (ctypes.c_int, [_ctx_p]),
    "lbm_adjoint_step": (ctypes.c_int, [_ctx_p, _vp, _vp, _vp, _vp, _vp]),
    "lbm_adjoint_steps": (ctypes.c_int, [_ctx_p, ctypes.c_int, _vp, _vp, _vp, _vp, _vp]),
    "lbm_adjoint_steps_noalloc": (ctypes.c_int, [_ctx_p, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "lbm_strain_loss_seed": (ctypes.c_int, [_ctx_p, _vp, _vp, ctypes.POINTER(ctypes.c_double), _vp]),
    "lbm_init_adjoint": (ctypes.c_int, [_ctx_p, _vp, _vp, _vp, _vp]),
    "lbm_destroy": (None, [_ctx_p]),
    "lbm_stream_copy": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp]),
    "lbm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "lbm_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
if _lib.lbm_params_size() != ctypes.sizeof(lbm_params):
    raise ImportError(f"{_LIB_PATH}: lbm_params is {_lib.lbm_params_size()} bytes in the library, "
                      f"{ctypes.sizeof(lbm_params)} in this binding; rebuild the library")


class LBMError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.lbm_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.lbm_status_string(status).decode()} ({msg})")
        self.status = status


def _check(status: int, where: str) -> int:
    if status != LBM_OK:
        raise LBMError(status, where)
    return status


def library_path() -> str:
    return str(_LIB_PATH)


def _ptr(t) -> Optional[int]:
    """Device pointer of a tensor (or None / a raw integer address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


@dataclass
class Params:
    """Python mirror of lbm_params (defaults: D3Q19, FP32, tau_nu = 0.8 rates)."""

    nx: int
    ny: int
    nz: int = 1
    lattice: int = LBM_D3Q19
    storage: int = LBM_F32
    walls_y: int = 0
    rho0: float = 1.0
    s: Sequence[float] = field(default_factory=lambda: [0.0] * 19)
    omega_eps: float = 3.0
    omega_epsj: float = -5.5
    omega_xx: float = -0.5
    visc_kind: int = LBM_VISC_CONST
    visc_strain: int = LBM_STRAIN_YU
    nu0: float = 0.0
    c_smag: float = 0.1
    K_pl: float = 0.1
    n_pl: float = 1.0
    nu_min: float = 1e-3
    nu_max: float = 1.0
    force: Sequence[float] = (0.0, 0.0, 0.0)
    force_field: object = None  # device tensor (3*N float32) or None
    strain_force_correction: int = 0

    def to_c(self) -> lbm_params:
        p = lbm_params()
        p.lattice, p.storage = self.lattice, self.storage
        p.nx, p.ny, p.nz, p.walls_y = self.nx, self.ny, self.nz, int(self.walls_y)
        p.rho0 = self.rho0
        ss = list(self.s) + [0.0] * (19 - len(self.s))
        for k in range(19):
            p.s[k] = float(ss[k])
        p.omega_eps, p.omega_epsj, p.omega_xx = self.omega_eps, self.omega_epsj, self.omega_xx
        p.visc_kind, p.visc_strain = self.visc_kind, self.visc_strain
        p.nu0, p.c_smag, p.K_pl, p.n_pl = self.nu0, self.c_smag, self.K_pl, self.n_pl
        p.nu_min, p.nu_max = self.nu_min, self.nu_max
        for a in range(3):
            p.force[a] = float(self.force[a])
        p.force_field = _ptr(self.force_field)
        p.strain_force_correction = int(self.strain_force_correction)
        return p

    @property
    def q(self) -> int:
        return self.lattice

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz


# --- the C ABI, name for name ---------------------------------------------------------------

def lbm_population_bytes(params: Params) -> int:
    return int(_lib.lbm_population_bytes(ctypes.byref(params.to_c())))


def lbm_init(params: Params, f_a, f_b, s_nu_field=None, rho_u=None, grad_u=None, stream=None) -> int:
    ctx = _ctx_p()
    cp = params.to_c()
    _check(_lib.lbm_init(ctypes.byref(ctx), ctypes.byref(cp), _ptr(f_a), _ptr(f_b), _ptr(s_nu_field),
                         _ptr(rho_u), _ptr(grad_u), _stream(stream)), "lbm_init")
    return ctx.value


def lbm_step(ctx: int, nsteps: int = 1, S_out=None, strain_kind: int = LBM_STRAIN_YU, save=None, stream=None):
    _check(_lib.lbm_step(ctx, int(nsteps), _ptr(S_out), int(strain_kind), _ptr(save), _stream(stream)), "lbm_step")


def lbm_strain(ctx: int, strain_kind: int, S_out, stream=None):
    _check(_lib.lbm_strain(ctx, int(strain_kind), _ptr(S_out), _stream(stream)), "lbm_strain")


def lbm_reduce(ctx: int, stream=None, allow_nonfinite: bool = False):
    out = (ctypes.c_double * 8)()
    st = _lib.lbm_reduce(ctx, out, _stream(stream))
    if not (allow_nonfinite and st == LBM_ENONFINITE):
        _check(st, "lbm_reduce")
    return list(out)


def lbm_reduce_async(ctx: int, out, stream=None):
    """Queue the diagnostics into ``out`` (8 float64: a device tensor or a pinned host
    tensor); read it after the stream has passed this point."""
    _check(_lib.lbm_reduce_async(ctx, _ptr(out), _stream(stream)), "lbm_reduce_async")


def lbm_get_populations(ctx: int, f_canon, stream=None):
    _check(_lib.lbm_get_populations(ctx, _ptr(f_canon), _stream(stream)), "lbm_get_populations")


def lbm_set_populations(ctx: int, f_canon, stream=None):
    _check(_lib.lbm_set_populations(ctx, _ptr(f_canon), _stream(stream)), "lbm_set_populations")


def lbm_state_bytes(ctx: int) -> int:
    return int(_lib.lbm_state_bytes(ctx))


def lbm_save_state(ctx: int, dst, stream=None):
    _check(_lib.lbm_save_state(ctx, _ptr(dst), _stream(stream)), "lbm_save_state")


def lbm_load_state(ctx: int, src, stream=None):
    _check(_lib.lbm_load_state(ctx, _ptr(src), _stream(stream)), "lbm_load_state")


def lbm_step_count(ctx: int) -> int:
    return int(_lib.lbm_step_count(ctx))


def lbm_set_step_count(ctx: int, n: int):
    _check(_lib.lbm_set_step_count(ctx, int(n)), "lbm_set_step_count")


def lbm_save_planes(ctx: int) -> int:
    return int(_lib.lbm_save_planes(ctx))


def lbm_adjoint_planes(ctx: int) -> int:
    return int(_lib.lbm_adjoint_planes(ctx))


def lbm_adjoint_step(ctx: int, rec_n, lam_in, lam_out, grad_force=None, stream=None):
    _check(_lib.lbm_adjoint_step(ctx, _ptr(rec_n), _ptr(lam_in), _ptr(lam_out), _ptr(grad_force), _stream(stream)),
           "lbm_adjoint_step")


def lbm_adjoint_steps(ctx: int, nsteps: int, rec, lam_a, lam_b, grad_force=None, stream=None):
    _check(_lib.lbm_adjoint_steps(ctx, int(nsteps), _ptr(rec), _ptr(lam_a), _ptr(lam_b), _ptr(grad_force),
                                  _stream(stream)), "lbm_adjoint_steps")


def lbm_adjoint_steps_noalloc(ctx: int, nsteps: int, rec, lam, grad_force=None, stream=None):
    _check(_lib.lbm_adjoint_steps_noalloc(ctx, int(nsteps), _ptr(rec), _ptr(lam), _ptr(grad_force), _stream(stream)),
           "lbm_adjoint_steps_noalloc")


def lbm_strain_loss_seed(ctx: int, lam_out, grad_force=None, stream=None) -> float:
    J = ctypes.c_double(0.0)
    _check(_lib.lbm_strain_loss_seed(ctx, _ptr(lam_out), _ptr(grad_force), ctypes.byref(J), _stream(stream)),
           "lbm_strain_loss_seed")
    return J.value


def lbm_init_adjoint(ctx: int, rho_u, lam0, grad_u0, stream=None):
    _check(_lib.lbm_init_adjoint(ctx, _ptr(rho_u), _ptr(lam0), _ptr(grad_u0), _stream(stream)), "lbm_init_adjoint")


def lbm_destroy(ctx: int):
    _lib.lbm_destroy(ctx)


def lbm_stream_copy(src, dst, nbytes: int, stream=None):
    _check(_lib.lbm_stream_copy(_ptr(src), _ptr(dst), int(nbytes), _stream(stream)), "lbm_stream_copy")


def lbm_status_string(status: int) -> str:
    return _lib.lbm_status_string(int(status)).decode()


def lbm_last_error() -> str:
    return _lib.lbm_last_error().decode()
