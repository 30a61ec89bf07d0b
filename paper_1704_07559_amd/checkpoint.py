"""Checkpoint / resume and a guarded run loop around the C ABI.

* ``save_checkpoint`` / ``load_checkpoint``: the context's state (internal population buffer
  and, for the lagged viscosity models, the s_nu field, as lbm_save_state writes it), the step
  counter and the parameters, in one file readable with ``torch.load(weights_only=True)``.
  The kernels are deterministic, so a resumed run continues bit-identically.
* ``run_guarded``: advance in chunks, check the FP64 diagnostics (lbm_reduce) after each
  chunk, keep a device-side snapshot of the last state that passed, and on a non-finite state
  or a velocity above a Mach watchdog restore that snapshot and raise ``Diverged``.

Host-side bookkeeping only; every step and every check runs in the library's kernels.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import torch

from . import capi
from .lbm import LBM

FORMAT = 1


class Diverged(RuntimeError):
    """The state became non-finite or too fast; the context was rolled back to ``step``."""

    def __init__(self, step: int, reason: str, diagnostics: dict):
        super().__init__(f"state rejected ({reason}); rolled back to step {step}")
        self.step = step
        self.reason = reason
        self.diagnostics = diagnostics


def _params_dict(p: capi.Params) -> dict:
    d = {f.name: getattr(p, f.name) for f in dataclasses.fields(p) if f.name != "force_field"}
    d["s"] = [float(v) for v in d["s"]]
    d["force"] = [float(v) for v in d["force"]]
    return d


def save_checkpoint(sim: LBM, path) -> None:
    state = sim.save_state()
    ff = sim.params.force_field
    torch.save({"format": FORMAT, "params": _params_dict(sim.params),
                "force_field": None if ff is None else ff.detach().cpu(),
                "step": int(sim.step_count), "state": state.cpu()}, path)


def load_checkpoint(path, device: str = "cuda") -> LBM:
    d = torch.load(path, map_location="cpu", weights_only=True)
    if d.get("format") != FORMAT:
        raise ValueError(f"{path}: unknown checkpoint format {d.get('format')}")
    p = capi.Params(**d["params"])
    if d["force_field"] is not None:
        p.force_field = d["force_field"].to(device).contiguous()
    sim = LBM(p, device=device)
    state = d["state"].to(device)
    if state.numel() != capi.lbm_state_bytes(sim.ctx):
        sim.close()
        raise ValueError(f"{path}: state size does not match its parameters")
    sim.load_state(state)
    capi.lbm_set_step_count(sim.ctx, d["step"])
    torch.cuda.current_stream().synchronize()
    return sim


def run_guarded(sim: LBM, nsteps: int, check_every: int = 100, umax_limit: float = 0.4,
                after_chunk: Optional[Callable[[LBM, int], None]] = None) -> dict:
    """Advance ``nsteps`` steps in chunks of ``check_every``. After each chunk (and the
    optional ``after_chunk(sim, step)`` hook) the diagnostics are checked: a non-finite
    population or max |u| above ``umax_limit`` (a Mach watchdog; c_s = 0.577 in lattice
    units) restores the snapshot of the last accepted state and raises ``Diverged``.
    Returns the last accepted diagnostics."""
    last = sim.reduce(allow_nonfinite=True)
    if last["nonfinite"]:
        raise ValueError("the starting state is not finite")
    snap = sim.save_state()
    snap_step = sim.step_count
    done = 0
    while done < nsteps:
        k = min(check_every, nsteps - done)
        sim.step(k)
        done += k
        if after_chunk is not None:
            after_chunk(sim, sim.step_count)
        diag = sim.reduce(allow_nonfinite=True)
        reason = None
        if diag["nonfinite"]:
            reason = f"{diag['nonfinite']} non-finite populations"
        elif not diag["umax"] <= umax_limit:
            reason = f"max |u| = {diag['umax']:.3g} above {umax_limit}"
        if reason is not None:
            sim.load_state(snap)
            capi.lbm_set_step_count(sim.ctx, snap_step)
            torch.cuda.current_stream().synchronize()
            raise Diverged(snap_step, reason, diag)
        capi.lbm_save_state(sim.ctx, snap)
        snap_step = sim.step_count
        last = diag
    return last
