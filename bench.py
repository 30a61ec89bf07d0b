#!/usr/bin/env python3
"""Throughput of the fused D3Q19 MRT collide-stream-strain step on one MI355X.

Workload (the headline configuration): D3Q19 He-Luo MRT LES on a 256^3 periodic box,
FP32 populations, Smagorinsky eddy viscosity (C_s = 0.1) driven by the Yu strain of every
node, initial velocity a seeded random solenoidal field with spectrum k^4 exp(-2 (k/4)^2)
and u_rms = 0.04 (seed 1704). One step = one launch of the fused kernel (pull streaming,
moments, equilibrium, Yu strain, Smagorinsky s_nu, relaxation, back-transform, store) over
all 16.8 M nodes; the FP64 diagnostics reduction (mass, momentum, energy, strain, max |u|,
non-finite watchdog) runs after every 100 steps, inside the timed region (a run of fewer steps
has none inside and is checked once after the timing).

Output: one JSON line. ``value`` is MLUPS (million lattice-node updates per second) with
inputs resident in HBM, over exactly --steps timed steps after --warmup untimed ones (the
device is first kept busy for a quarter second with STREAM-style copies, so the run does not
start from an idle GPU). ``roofline`` prices the step kernel's algorithmic bytes per node
(19 reads + 19 writes of 4 B, plus the 4 B read and write of the lagged s_nu field) against
the 8 TB/s HBM peak; its kernel time is the device time of all timed launches (HIP events
on the launch stream around every run of launches between two diagnostics), divided by the
number of launches. ``extra`` carries the other workloads (FP16/BF16-stored 384^3 runs and
their FP32 reference, the one-rank slab, implicit Smagorinsky, D3Q15, D2Q9 in FP32 and FP16
one and two steps per launch, the power-law channel, the adjoint, the Yu/Chai cost comparison
of Section 5.2): each is warmed up for at
least 0.2 s and timed over at least 0.25 s, whatever --steps is. ``cpu_baseline`` times the
FP64 oracle, single-threaded, on a bounded slab of the same workload and on the full 32^3
Taylor-Green parity run.

    python bench.py [--gpus 1] [--steps 1000] [--warmup 20]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time
from contextlib import nullcontext
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS & % HBM roofline, D3Q19 MRT+strain, FP32 vs FP16-stored; adjoint/fwd cost"
# The sources the D3Q19 step kernel is compiled from (launch.h holds host-side
# declarations only and is left out).
KERNEL_SOURCES = ["paper_1704_07559_amd/csrc/kernels_d3q19_step.hip", "paper_1704_07559_amd/csrc/d3q19_node.h",
                  "paper_1704_07559_amd/csrc/d3q19.h", "paper_1704_07559_amd/csrc/internal.h",
                  "paper_1704_07559_amd/csrc/codec.h", "paper_1704_07559_amd/csrc/static_for.h"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ... and, with the strain query kernel, those of the Section 5.2 comparison
STRAIN_SOURCES = KERNEL_SOURCES + ["paper_1704_07559_amd/csrc/kernels_d3q19.hip"]


def kernel_source_sha(sources=None) -> str:
    h = hashlib.sha256()
    for rel in sources or KERNEL_SOURCES:
        h.update((ROOT / rel).read_bytes())
    return h.hexdigest()[:16]


def read_traffic(name: str, sha: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel source (else None)."""
    f = ROOT / "profiles" / f"traffic_{name}.txt"
    if not f.exists():
        return None
    kv = {}
    for line in f.read_text().splitlines():
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != sha:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# VALU issue ceiling: one wave64 FP32 instruction takes 4 cycles on a SIMD (packed FP32 is
# off), 256 CUs x 4 SIMDs at 2.4 GHz.
VALU_WAVE_INSTS_PER_S = 256 * 4 * 2.4e9 / 4


def read_valu(label: str, sha: str):
    """VALU instructions per launch of the step kernel from the committed rocprofv3 counter
    summary (profiles/valu_step_d3q19_les.txt), if it was taken on the current kernel
    source (else None)."""
    f = ROOT / "profiles" / "valu_step_d3q19_les.txt"
    if not f.exists():
        return None
    kv = {}
    for line in f.read_text().splitlines():
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != sha:
        return None
    try:
        return float(kv[f"{label}_valu_insts"])
    except (KeyError, ValueError):
        return None


def valu_frac(insts, kernel_s):
    """Fraction of the chip's VALU issue rate the kernel used (None without counts)."""
    return None if insts is None else round(insts / kernel_s / VALU_WAVE_INSTS_PER_S, 4)


def _workloads():
    from paper_1704_07559_amd import workloads
    return workloads


def rates(tau_nu):
    """D3Q19 rates of the workloads (d'Humieres values, s_nu = 1/tau_nu in slots 9, 11, 13,
    14, 15; paper_1704_07559_amd/configs records them per workload)."""
    return _workloads().rates_d3q19(tau_nu)


def rates15(tau_nu):
    """D3Q15 rates (rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, p_ww, p_xy, p_yz, p_xz,
    m_xyz): s_e = 1.6, s_eps = 1.2, s_q = 1.6, s_m = 1.2 (d'Humieres et al. 2002), s_nu = 1/tau_nu."""
    return _workloads().rates_d3q15(tau_nu)


def les_params(capi, n, storage):
    """The LES workload (configs/c1_les256.json; with FP16/BF16 storage the 384^3 one,
    configs/c3_les384_half.json) on an n^3 box."""
    w = _workloads()
    name = {capi.LBM_F32: "f32", capi.LBM_F16: "f16", capi.LBM_BF16: "bf16"}[storage]
    return w.params(w.load("C1" if name == "f32" else "C3"), storage=name, grid={"nx": n, "ny": n, "nz": n})


def settle(torch, capi, seconds=0.25):
    """Keep the device busy with STREAM-style copies of 256 MiB for ``seconds`` before a timed
    leg, so that it does not start from a GPU left idle by host-side setup."""
    a = torch.empty(1 << 26, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            capi.lbm_stream_copy(a, b, a.numel() * 4, stream)
        torch.cuda.synchronize()
    del a, b


def time_run(sim, steps, warmup, reduce_every=100, windows=None, min_warm_s=0.0, min_span_s=0.0):
    """Run ``warmup`` untimed steps, then a timed run; returns a dict with the wall time, the
    kernel time per launch, the number of timed steps and checks, and the last diagnostics.

    ``min_warm_s``: keep warming up (in runs of 10 steps) until that much wall time has passed.
    ``min_span_s``: lengthen the timed run to at least that much device time (estimated from 10
    launches), so that the measurement does not depend on ``steps`` being large.
    The diagnostics run after every ``reduce_every`` steps inside the timed region, without
    stalling the stream (lbm_reduce_async into pinned host slots, read once the run has
    finished); a run shorter than that has none inside, and is checked once after the timing.
    HIP events on the launch stream bracket every run of launches between two reductions; the
    kernel time is their summed device time over the number of launches (the reductions are
    outside the brackets, the gaps between back-to-back launches inside). ``windows`` (a list)
    receives the device time per step (ms) of each full window."""
    import torch
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    extra_warm = 0
    while time.perf_counter() - t0 < min_warm_s:
        sim.step(10)
        extra_warm += 10
        torch.cuda.synchronize()
    if min_span_s > 0.0:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.step(10)
        e1.record()
        torch.cuda.synchronize()
        extra_warm += 10
        est = e0.elapsed_time(e1) / 1e3 / 10
        steps = max(steps, int(math.ceil(min_span_s / est)))
    bounds = list(range(0, steps, reduce_every)) + [steps]
    chunks = list(zip(bounds[:-1], bounds[1:]))
    checks = steps // reduce_every
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in chunks]
    slots = torch.zeros((max(checks, 1), 8), dtype=torch.float64, pin_memory=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, ((a, b), (e0, e1)) in enumerate(zip(chunks, ev)):
        e0.record()
        sim.step(b - a)
        e1.record()
        if b - a == reduce_every:
            sim.reduce_async(slots[c])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev = [e0.elapsed_time(e1) / 1e3 for e0, e1 in ev]
    kern = sum(dev) / steps
    if windows is not None:
        for (a, b), d in zip(chunks, dev):
            if b - a == reduce_every:
                windows.append(d * 1e3 / reduce_every)
    bad = [i for i in range(checks) if slots[i, 7].item() != 0.0]
    if bad:
        log(f"non-finite populations at check {bad[0]} (step {chunks[bad[0]][1]})")
    last = sim.diagnostics(slots[checks - 1].tolist()) if checks == len(chunks) else sim.reduce(allow_nonfinite=True)
    return {"wall": wall, "kernel_s": kern, "steps": steps, "warmup": warmup + extra_warm, "checks": checks,
            "diag": last}


# Extra legs: untimed warm-up of at least 0.2 s and a timed span of at least 0.25 s of device
# time, whatever --steps and --warmup are.
LEG_WARM_S = 0.2
LEG_SPAN_S = 0.25


def leg(torch, capi, sim, nodes, steps, warmup, bytes_per_node, **extra):
    """Time one extra workload (settled device, minimum warm-up and span) and summarise it."""
    settle(torch, capi)
    r = time_run(sim, steps, warmup, min_warm_s=LEG_WARM_S, min_span_s=LEG_SPAN_S)
    out = {"MLUPS": round(nodes * r["steps"] / r["wall"] / 1e6, 1),
           "ms_per_step": round(r["wall"] / r["steps"] * 1e3, 4),
           "kernel_ms": round(r["kernel_s"] * 1e3, 4), "bytes_per_node": bytes_per_node,
           "hbm_frac": round(bytes_per_node * nodes / r["kernel_s"] / 1e9 / HBM_PEAK_GBS, 4),
           "steps": r["steps"], "warmup": r["warmup"], "checks": r["checks"],
           "ke": r["diag"]["ke"], "nonfinite": r["diag"]["nonfinite"]}
    out.update(extra)
    return out, r


def step_kernel_name(nx, ny, storage="f32", walls=False, corrected=False):
    """The D3Q19 step kernel instance the library launches for a box (its launch rule restated:
    rows split into segments of the widest power of two <= 256 dividing nx when nx is a
    multiple of 64, else one masked segment; pull mode 2 (whole rows, LDS exchange) when one
    block holds whole rows of >= 64 nodes and its rows tile ny, 1 when a segment covers the
    row, 0 for part rows)."""
    tx = 256
    if nx % 64 == 0:
        while nx % tx:
            tx //= 2
    else:
        tx = 1
        while tx < nx and tx < 256:
            tx *= 2
    py = 1
    while py < ny:
        py *= 2
    ty = min(256 // tx, py)
    mode = 2 if (tx == nx and tx >= 64 and ny % ty == 0) else (1 if tx >= nx else 0)
    st = {"f32": "float", "f16": "_Float16", "bf16": "__bf16"}[storage]
    return f"lbm::d3q19::step_kernel<{st}, {str(walls).lower()}, {mode}, {str(corrected).lower()}>"


def channel_runs(torch, capi, lbm, steps, warmup):
    """Power-law channel 128 x 128 x 512 (walls at y = -1/2 and 127.5, periodic x and z),
    uniform body force 1e-6 along z, viscosity from the Chai strain, FP32, from rest; one
    run per index n. Algorithmic bytes per node: 160 (populations + lagged s_nu)."""
    out = {}
    w = _workloads()
    cfg = w.load("C2")
    nx, ny, nz = cfg["grid"]["nx"], cfg["grid"]["ny"], cfg["grid"]["nz"]
    N = nx * ny * nz
    for n_pl in cfg["viscosity"]["n_pl"]:
        sim = lbm.LBM(w.params(cfg, n_pl=n_pl))
        log(f"power-law channel n={n_pl}")
        o, r = leg(torch, capi, sim, N, steps, warmup, 160, umax=None,
                   kernel=step_kernel_name(nx, ny, walls=True))
        o["umax"] = r["diag"]["umax"]
        sim.close()
        out[f"n{n_pl}"] = o
    torch.cuda.empty_cache()
    return out


def _event_time(torch, fn, reps):
    """Mean device time of fn() over reps back-to-back calls (events on the current stream),
    after one untimed call."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


# Section 5.2 counts the operations of one node's strain: Chai's formula 957 multiplications
# and 792 additions, Yu's 155 and 113 (dense 19 x 19 products).
PAPER_OPS = {"yu": 155 + 113, "chai": 957 + 792}


def strain_formulas(torch, np, capi, lbm, u, reps, sha):
    """Yu against Chai on the chip (the operation counts of Section 5.2): on the 256^3 LES state,
    the strain query (lbm_strain, 76 + 4 B read, 24 B written per node) with either formula,
    the LES step emitting either strain every step (160 + 24 B), and the LES step whose
    viscosity is driven by either formula without emitting it (160 B). Device time per call
    over ``reps`` back-to-back calls; VALU instructions per wave from the committed counter
    summary (profiles/valu_strain_formulas.txt) when it was taken on the current kernels."""
    n = u.shape[1]
    N = n ** 3
    out = {}
    rho_u = lbm.rho_u_field(np.zeros((n, n, n)), u)
    sims = {}
    for drive, kind in (("yu", capi.LBM_STRAIN_YU), ("chai", capi.LBM_STRAIN_CHAI)):
        p = les_params(capi, n, capi.LBM_F32)
        p.visc_strain = kind
        sims[drive] = lbm.LBM(p, rho_u)
    del rho_u
    S = torch.empty((6, n, n, n), device="cuda")
    yu = sims["yu"]
    settle(torch, capi)
    yu.step(20)
    t = {}
    for name, kind in (("yu", capi.LBM_STRAIN_YU), ("chai", capi.LBM_STRAIN_CHAI)):
        t[f"query_{name}"] = _event_time(torch, lambda k=kind: capi.lbm_strain(yu.ctx, k, S), reps)
    for name, kind in (("yu", capi.LBM_STRAIN_YU), ("chai", capi.LBM_STRAIN_CHAI)):
        t[f"step_emit_{name}"] = _event_time(torch, lambda k=kind: yu.step(1, S_out=S, strain_kind=k), reps)
    for name in ("yu", "chai"):
        sims[name].step(20)
        t[f"step_drive_{name}"] = _event_time(torch, lambda s=sims[name]: s.step(1), reps)
    for s_ in sims.values():
        s_.close()
    del S, sims
    torch.cuda.empty_cache()
    bpn = {"query": 104, "step_emit": 184, "step_drive": 160}
    valu = read_valu_strain(sha)
    for key, sec in t.items():
        kind = key.rsplit("_", 1)[0]
        out[key] = {"kernel_ms": round(sec * 1e3, 4), "bytes_per_node": bpn[kind],
                    "hbm_frac": round(bpn[kind] * N / sec / 1e9 / HBM_PEAK_GBS, 4)}
        if valu and key in valu:
            out[key]["valu_per_wave"] = round(valu[key], 1)
    ratios = {}
    for kind in ("query", "step_emit", "step_drive"):
        r = {"time": round(t[f"{kind}_chai"] / t[f"{kind}_yu"], 4)}
        if valu and f"{kind}_chai" in valu and f"{kind}_yu" in valu:
            r["valu"] = round(valu[f"{kind}_chai"] / valu[f"{kind}_yu"], 4)
        ratios[kind] = r
    out["chai_over_yu"] = ratios
    out["paper_ops_per_node"] = {"yu": PAPER_OPS["yu"], "chai": PAPER_OPS["chai"],
                                 "chai_over_yu": round(PAPER_OPS["chai"] / PAPER_OPS["yu"], 4)}
    return out


def read_valu_strain(sha: str):
    """VALU instructions per wave of the Section 5.2 comparison kernels from the committed
    counter summary, if it was taken on the current kernel source (else None)."""
    f = ROOT / "profiles" / "valu_strain_formulas.txt"
    if not f.exists():
        return None
    kv = {}
    for line in f.read_text().splitlines():
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != sha:
        return None
    out = {}
    for k, v in kv.items():
        if k.endswith("_valu_per_wave"):
            try:
                out[k[: -len("_valu_per_wave")]] = float(v)
            except ValueError:
                pass
    return out or None


class SingleSteps:
    """A simulation stepped one lbm_step call (one launch) per step: the single-step path of
    a lattice whose lbm_step groups steps, for comparison."""

    def __init__(self, sim):
        self.sim = sim

    def step(self, nsteps=1):
        for _ in range(nsteps):
            self.sim.step(1)

    def __getattr__(self, name):
        return getattr(self.sim, name)


def other_kernels(torch, np, synth, capi, lbm, u, reps, steps, warmup):
    """The remaining kernels of the path, each against its algorithmic bytes per node: the
    diagnostics reduction (76 + 4 B read) on the 256^3 LES state, and the D2Q9 LES step on
    4096^2 (9 x 4 x 2 + 8 = 80 B per launch; 44 with FP16 storage), one launch per step and two
    steps per launch."""
    out = {}
    n = u.shape[1]
    N = n ** 3
    sim = lbm.LBM(les_params(capi, n, capi.LBM_F32), lbm.rho_u_field(np.zeros((n, n, n)), u))
    sim.step(warmup)
    t = _event_time(torch, lambda: sim.reduce(), 20)
    out["diagnostics_reduce_256"] = {"call_ms": round(t * 1e3, 4), "bytes_per_node": 80,
                                     "hbm_frac": round(80 * N / t / 1e9 / HBM_PEAK_GBS, 4),
                                     "note": "includes the final pass and the host copy"}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    m = 4096
    u2 = synth.spectrum_velocity((1, m, m), seed=1704, u_rms=0.04)[:2]
    w = _workloads()
    for name, storage, bpn in (("d2q9_les_4096sq", capi.LBM_F32, 80), ("d2q9_les_4096sq_f16", capi.LBM_F16, 44)):
        p2 = w.params(w.load("C1"), lattice="D2Q9", grid={"nx": m, "ny": m, "nz": 1})
        p2.storage = storage
        s2 = lbm.LBM(p2, lbm.rho_u_field(np.zeros((1, m, m)), u2))
        log(f"D2Q9 {m}^2 LES ({name}), one launch per step")
        single, _ = leg(torch, capi, SingleSteps(s2), m * m, steps, warmup, bpn)
        log(f"D2Q9 {m}^2 LES ({name}), two steps per launch")
        out[name], _ = leg(torch, capi, s2, m * m, steps, warmup, bpn // 2,
                           note=f"lbm_step takes D2Q9 steps two per launch: {bpn} B per node per launch, "
                                f"{bpn // 2} per step; kernel_ms per step")
        out[name]["one_launch_per_step"] = single
        out[name]["speedup"] = round(out[name]["MLUPS"] / single["MLUPS"], 3)
        s2.close()
        torch.cuda.empty_cache()
    return out


def copy_bandwidth(torch, capi):
    """Device-to-device copies of 1 GiB (1 GiB read + 1 GiB written), for context: the
    library's STREAM-style copy kernel (16-byte nontemporal accesses; the practical ceiling
    of a read-once/write-once pattern) and the runtime's own copy. GB/s of read + write."""
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    out = {}
    for name, fn in (("stream_copy_GBps", lambda: capi.lbm_stream_copy(a, b, a.numel() * 4, stream)),
                     ("runtime_copy_GBps", lambda: b.copy_(a))):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        out[name] = round(2 * (1 << 30) / (e0.elapsed_time(e1) / 1e3 / reps) / 1e9, 1)
    assert torch.equal(a, b)
    del a, b
    torch.cuda.empty_cache()
    return out


def adjoint_run(torch, np, synth, capi, lbm, warmup, visc="const"):
    """Strain-squared loss gradient on the 128^3 workload (configs/c4_adjoint128.json: seeded
    spectrum velocity, uniform random force U(-1e-6, 1e-6), tau_nu = 0.8, 500 steps,
    checkpoint every 50): wall time of
    the forward pass and of the backward pass (recompute + adjoint); the same with every
    step's record kept by the forward sweep (no recompute; the gradient must come out with
    the same bits); and the adjoint kernel alone against HBM (per step of a multi-step sweep,
    and as one step on canonical planes). Algorithmic bytes per node of the adjoint kernel: 200 for a constant
    viscosity (76 lambda in, 76 out, 12 j, 12 F, 24 grad_F); with visc="smagorinsky" (lagged,
    C_s = 0.1 on top of nu0 = 0.1) 236 (+ 28 for the 7 extra record planes, + 8 for the
    s_nu-field adjoint in and out)."""
    from paper_1704_07559_amd import autograd as ag
    w = _workloads()
    cfg = w.load("C4")
    n, nsteps, every = cfg["grid"]["nx"], cfg["steps"], cfg["checkpoint_every"]
    shape = (n, n, n)
    log(f"adjoint {n}^3 ({visc}): {nsteps} steps, checkpoint every {every}")
    ini, frc = cfg["init"], cfg["force"]
    u0 = torch.as_tensor(synth.spectrum_velocity(shape, seed=ini["seed"], u_rms=ini["u_rms"], k0=ini["k0"])
                         .astype(np.float32)).cuda()
    F = torch.as_tensor(synth.uniform_random_force(shape, seed=frc["seed"], amp=frc["amplitude"])
                        .astype(np.float32)).cuda()
    p = w.params(cfg)
    bpn = 200
    if visc == "smagorinsky":
        p.visc_kind, p.nu0, p.c_smag = capi.LBM_VISC_SMAGORINSKY, w.nu_of_tau(cfg["tau_nu"]), 0.1
        bpn = 236
    # warm-up on a short problem (kernel loading, allocator)
    u_w, F_w = u0.clone().requires_grad_(True), F.clone().requires_grad_(True)
    ag.strain_loss(u_w, F_w, ag.StrainLossProblem(p, 2 * every, every)).backward()
    u0.requires_grad_(True)
    F.requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = ag.strain_loss(u0, F, ag.StrainLossProblem(p, nsteps, every))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    gu_ck, gF_ck = u0.grad.clone(), F.grad.clone()
    # the same gradient with every step's record kept by the forward sweep (no recompute;
    # 12 or 40 bytes per node and step of HBM)
    u0.grad, F.grad = None, None
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    Jr = ag.strain_loss(u0, F, ag.StrainLossProblem(p, nsteps, every, record_all=True))
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    Jr.backward()
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    same = bool(Jr.item() == J.item() and torch.equal(u0.grad, gu_ck) and torch.equal(F.grad, gF_ck))
    torch.cuda.empty_cache()
    # adjoint kernel alone, as the backward sweep runs it: lbm_adjoint_steps over the record
    # of K steps (the intermediate adjoint states row-interleaved), device time per step over
    # at least a quarter second; and one lbm_adjoint_step on canonical planes
    N = n ** 3
    p.force_field = F.detach().reshape(3, N)
    sim = lbm.LBM(p)
    K = 10
    jb = torch.zeros((K, sim.save_planes, N), device="cuda")
    sim.step(K, save=jb)
    la = torch.randn((sim.adjoint_planes, N), device="cuda")
    lb = torch.empty_like(la)
    gF = torch.zeros((3, N), device="cuda")
    sweep = lambda: capi.lbm_adjoint_steps(sim.ctx, K, jb, la, lb, gF)
    est = _event_time(torch, sweep, 3)
    k_adj = _event_time(torch, sweep, max(5, math.ceil(0.25 / est))) / K
    single = lambda: capi.lbm_adjoint_step(sim.ctx, jb[0], la, lb, gF)
    k_one = _event_time(torch, single, max(50, math.ceil(0.25 / (est / K))))
    sim.close()
    fwd, bwd = t1 - t0, t2 - t1
    fwd_r, bwd_r = t4 - t3, t5 - t4
    return {"J": J.item(), "forward_s": round(fwd, 4), "backward_s": round(bwd, 4),
            "backward_over_forward": round(bwd / fwd, 3),
            "recorded": {"forward_s": round(fwd_r, 4), "backward_s": round(bwd_r, 4),
                         "backward_over_forward": round(bwd_r / fwd_r, 3),
                         "gradient_over_plain_forward": round((fwd_r + bwd_r) / fwd, 3),
                         "record_bytes": nsteps * (3 if visc == "const" else 10) * N * 4,
                         "same_gradient_bits": same},
            "adjoint_kernel_ms": round(k_adj * 1e3, 4), "adjoint_bytes_per_node": bpn,
            "adjoint_hbm_frac": round(bpn * N / k_adj / 1e9 / HBM_PEAK_GBS, 4),
            "adjoint_single_step_ms": round(k_one * 1e3, 4),
            "grad_u0_norm": float(u0.grad.norm()), "grad_F_norm": float(F.grad.norm())}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(u_full, n_slab=64, steps=6):
    """The FP64 oracle as it stands, on one host thread (its element-wise NumPy work runs on
    one core; more BLAS threads gain little): ``steps`` steps of a 256 x 256 x n_slab z-slab of
    the headline field (periodic in the slab, Smagorinsky from Yu), and the full 32^3 rotated
    Taylor-Green parity run (200 steps, both strains every step)."""
    import numpy as np

    import synth
    from oracle import d3q19 as od
    try:
        from threadpoolctl import threadpool_limits
    except Exception:   # pragma: no cover
        threadpool_limits = None
    u = np.ascontiguousarray(u_full[:, :n_slab])
    shape = u.shape[1:]
    tau0 = 0.51
    p = od.Params(s=od.default_rates(tau0), visc_kind="smagorinsky", visc_strain="yu", nu0=(tau0 - 0.5) / 3.0,
                  c_smag=0.1)
    sim = od.Simulation(p, od.init_populations(np.zeros(shape), u, p))
    c0 = (32, 32, 32)
    drho, u0, grad = synth.tgv_rotated(c0, u0=0.05)
    p0 = od.Params(s=od.default_rates(0.8))
    tgv = od.Simulation(p0, od.init_populations(drho, u0, p0, grad))
    with (threadpool_limits(limits=1) if threadpool_limits is not None else nullcontext()):
        t0 = time.perf_counter()
        sim.step(steps)
        dt = time.perf_counter() - t0
        t0 = time.perf_counter()
        tgv.step(200)
        dt0 = time.perf_counter() - t0
    nodes = int(np.prod(shape))
    return {"value": nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"FP64 NumPy oracle on one thread, {shape[2]}x{shape[1]}x{shape[0]} z-slab of the 256^3 "
                      f"workload, {steps} steps, {dt:.1f} s",
            "cpu_model": _cpu_model(),
            "c0_full_run": {"grid": "32^3 rotated Taylor-Green", "steps": 200, "seconds": round(dt0, 2),
                            "MLUPS": round(32 ** 3 * 200 / dt0 / 1e6, 3)}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="edge of the cubic LES box (default 256)")
    ap.add_argument("--no-extra", action="store_true", help="skip every workload but the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--storage-probe", choices=("f16", "bf16", "f32"),
                    help="only step the 384^3 LES in that storage (--steps steps; counter collection)")
    ap.add_argument("--slab-probe", action="store_true",
                    help="only step the 384x384x48 FP16 slab (--steps steps; counter collection)")
    ap.add_argument("--strain-probe", action="store_true",
                    help="only run the Section 5.2 kernels on the 256^3 LES state, 5 calls each in a fixed "
                         "order (counter collection)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration for rocprofv3)")
    ap.add_argument("--d2q9-probe", choices=("f32", "f16"),
                    help="only step the 4096^2 D2Q9 LES in that storage: 8 steps two per launch, then 4 "
                         "one per launch (counter collection)")
    ap.add_argument("--adjoint-probe", action="store_true",
                    help="only run three 6-step adjoint sweeps (lbm_adjoint_steps) on an --n^3 box, constant "
                         "viscosity then lagged Smagorinsky, after the forward steps that record them "
                         "(counter collection)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)

    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 4, "copy_probe_bytes_written": b.numel() * 4}))
        return

    import synth
    from paper_1704_07559_amd import capi, lbm

    if args.storage_probe or args.slab_probe:
        m = 384
        st = capi.LBM_F16 if args.slab_probe else {"f16": capi.LBM_F16, "bf16": capi.LBM_BF16,
                                                   "f32": capi.LBM_F32}[args.storage_probe]
        u3 = synth.spectrum_velocity((m, m, m), seed=1704, u_rms=0.04)
        p = les_params(capi, m, st)
        if args.slab_probe:
            p.nz = m // 8
            u3 = np.ascontiguousarray(u3[:, : m // 8])
        sim = lbm.LBM(p, lbm.rho_u_field(np.zeros(u3.shape[1:]), u3))
        del u3
        sim.step(args.warmup + args.steps)
        d = sim.reduce(allow_nonfinite=True)
        sim.close()
        print(json.dumps({"probe": "slab" if args.slab_probe else args.storage_probe,
                          "steps": args.warmup + args.steps, "nonfinite": d["nonfinite"]}))
        return

    if args.d2q9_probe:
        m = 4096
        w = _workloads()
        p2 = w.params(w.load("C1"), lattice="D2Q9", grid={"nx": m, "ny": m, "nz": 1})
        p2.storage = capi.LBM_F16 if args.d2q9_probe == "f16" else capi.LBM_F32
        u2 = synth.spectrum_velocity((1, m, m), seed=1704, u_rms=0.04)[:2]
        sim = lbm.LBM(p2, lbm.rho_u_field(np.zeros((1, m, m)), u2))
        sim.step(8)
        SingleSteps(sim).step(4)
        d = sim.reduce(allow_nonfinite=True)
        sim.close()
        print(json.dumps({"probe": "d2q9", "storage": args.d2q9_probe, "grouped_launches": 4, "single_launches": 4,
                          "nonfinite": d["nonfinite"]}))
        return

    if args.adjoint_probe:
        # the C4 recipe (seeded spectrum velocity, uniform random force field, tau_nu = 0.8) on
        # an n^3 box; the sweep's first step reads canonical planes and writes row-interleaved
        # states, its last reads them and writes canonical planes, the 4 between stay
        # row-interleaved
        w = _workloads()
        cfg = w.load("C4")
        n, K = args.n, 6
        N = n ** 3
        ini, frc = cfg["init"], cfg["force"]
        u = synth.spectrum_velocity((n, n, n), seed=ini["seed"], u_rms=ini["u_rms"], k0=ini["k0"])
        F = torch.as_tensor(synth.uniform_random_force((n, n, n), seed=frc["seed"], amp=frc["amplitude"])
                            .astype(np.float32)).cuda().reshape(3, N)
        for visc in ("const", "smagorinsky"):
            p = w.params(cfg, grid={"nx": n, "ny": n, "nz": n})
            if visc == "smagorinsky":
                p.visc_kind, p.nu0, p.c_smag = capi.LBM_VISC_SMAGORINSKY, w.nu_of_tau(cfg["tau_nu"]), 0.1
            p.force_field = F
            sim = lbm.LBM(p, lbm.rho_u_field(np.zeros((n, n, n)), u))
            rec = torch.empty((K, sim.save_planes, N), device="cuda")
            sim.step(K, save=rec)
            la = torch.randn((sim.adjoint_planes, N), device="cuda")
            lb = torch.empty_like(la)
            gF = torch.zeros((3, N), device="cuda")
            settle(torch, capi)
            for _ in range(3):
                capi.lbm_adjoint_steps(sim.ctx, K, rec, la, lb, gF)
            torch.cuda.synchronize()
            sim.close()
            del rec, la, lb, gF
            torch.cuda.empty_cache()
        print(json.dumps({"probe": "adjoint", "n": n, "steps": K, "sweeps": 3}))
        return

    if args.strain_probe:
        n = args.n
        u = synth.spectrum_velocity((n, n, n), seed=1704, u_rms=0.04)
        rho_u = lbm.rho_u_field(np.zeros((n, n, n)), u)
        del u
        sims = {}
        for drive, kind in (("yu", capi.LBM_STRAIN_YU), ("chai", capi.LBM_STRAIN_CHAI)):
            p = les_params(capi, n, capi.LBM_F32)
            p.visc_strain = kind
            sims[drive] = lbm.LBM(p, rho_u)
        S = torch.empty((6, n, n, n), device="cuda")
        # dispatch order (the counter summary splits the records by it): 5 queries Yu, 5 Chai,
        # 5 steps emitting Yu, 5 emitting Chai, 5 steps driven by Yu, 5 driven by Chai
        for kind in (capi.LBM_STRAIN_YU, capi.LBM_STRAIN_CHAI):
            for _ in range(5):
                capi.lbm_strain(sims["yu"].ctx, kind, S)
        for kind in (capi.LBM_STRAIN_YU, capi.LBM_STRAIN_CHAI):
            for _ in range(5):
                sims["yu"].step(1, S_out=S, strain_kind=kind)
        for drive in ("yu", "chai"):
            sims[drive].step(5)
        torch.cuda.synchronize()
        for s_ in sims.values():
            s_.close()
        print(json.dumps({"probe": "strain", "n": n}))
        return

    n = args.n
    ini = _workloads().load("C1")["init"]
    log(f"generating the {n}^3 initial field")
    u = synth.spectrum_velocity((n, n, n), seed=ini["seed"], u_rms=ini["u_rms"], k0=ini["k0"])
    rho_u = lbm.rho_u_field(np.zeros((n, n, n)), u)
    sim = lbm.LBM(les_params(capi, n, capi.LBM_F32), rho_u)
    del rho_u
    N = n ** 3
    log(f"FP32 {n}^3: {args.warmup} warmup + {args.steps} timed steps")
    settle(torch, capi)
    win = []
    r = time_run(sim, args.steps, args.warmup, windows=win)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    wall, kern, diag = r["wall"], r["kernel_s"], r["diag"]
    mlups = N * args.steps / wall / 1e6
    bytes_per_node = 19 * 4 * 2 + 4 * 2
    achieved = bytes_per_node * N / kern / 1e9
    sha = kernel_source_sha()
    traffic = read_traffic("step_d3q19_f32_les256", sha) if n == 256 else None  # taken on 256^3
    result = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"D3Q19 He-Luo MRT LES {n}^3 periodic, FP32 populations, Smagorinsky C_s=0.1 "
                               f"from the Yu strain, k^4 exp(-2(k/4)^2) spectrum seed 1704 u_rms 0.04, "
                               f"FP64 diagnostics after every 100 steps inside the timed region "
                               f"({r['checks']} in this run)",
                   "nodes": N, "lattice": "D3Q19", "storage": "f32"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": step_kernel_name(n, n),
                     "kernel_ms": round(kern * 1e3, 4), "kernel_time": "device time of all timed launches / launches",
                     "bytes_per_node": bytes_per_node, "kernel_source_sha": sha,
                     "valu_issue_frac": valu_frac(read_valu("f32_les256", sha) if n == 256 else None, kern)},
        "diagnostics": {"mass": diag["mass"], "ke": diag["ke"], "umax": diag["umax"], "nonfinite": diag["nonfinite"]},
    }
    if win:
        wm = sorted(N / (w * 1e-3) / 1e6 for w in win)
        result["windows_MLUPS"] = {"count": len(wm), "min": round(wm[0], 1), "median": round(wm[len(wm) // 2], 1),
                                   "max": round(wm[-1], 1)}

    if not args.no_extra:
        extra = {}
        K, W = args.steps, args.warmup
        cfg3 = _workloads().load("C3")
        m, ini3 = cfg3["grid"]["nx"], cfg3["init"]
        log(f"generating the {m}^3 initial field")
        u3 = synth.spectrum_velocity((m, m, m), seed=ini3["seed"], u_rms=ini3["u_rms"], k0=ini3["k0"])
        rho_u3 = lbm.rho_u_field(np.zeros((m, m, m)), u3)
        del u3
        for name, st, bpn in (("f16", capi.LBM_F16, 19 * 2 * 2 + 8), ("bf16", capi.LBM_BF16, 19 * 2 * 2 + 8),
                              ("f32", capi.LBM_F32, 19 * 4 * 2 + 8)):
            s3 = lbm.LBM(les_params(capi, m, st), rho_u3)
            log(f"{name} {m}^3")
            o, r3 = leg(torch, capi, s3, m ** 3, K, W, bpn, kernel=step_kernel_name(m, m, name))
            if name == "f16":
                o["valu_issue_frac"] = valu_frac(read_valu("f16_les384", sha), r3["kernel_s"])
            extra[f"les384_{name}"] = o
            s3.close()
            del s3
            torch.cuda.empty_cache()
        # one rank's share of a z-slab decomposition of the 384^3 FP16 run over 8 GPUs: the
        # 384 x 384 x 48 interior, updated by the same kernel (its faces wrap periodically
        # here; a decomposed run would read them from 2 ghost planes exchanged per step)
        zs = m // 8
        ps = les_params(capi, m, capi.LBM_F16)
        ps.nz = zs
        slab = rho_u3.reshape(4, m, m, m)[:, :zs].contiguous()
        ss = lbm.LBM(ps, slab)
        log(f"f16 {m}x{m}x{zs} slab")
        halo = 2 * 5 * m * m * 2  # the 5 populations with c_z = +1 and the 5 with c_z = -1, FP16
        extra["slab_384x384x48_f16"], _ = leg(torch, capi, ss, m * m * zs, K, W, 84, halo_bytes_per_step=halo,
                                              kernel=step_kernel_name(m, m, "f16"))
        ss.close()
        del ss, slab, rho_u3
        torch.cuda.empty_cache()
        # the same 256^3 LES with the implicit (non-lagged) Smagorinsky coupling: no s_nu field
        pi = les_params(capi, n, capi.LBM_F32)
        pi.visc_kind = capi.LBM_VISC_SMAGORINSKY_IMPLICIT
        si = lbm.LBM(pi, lbm.rho_u_field(np.zeros((n, n, n)), u))
        log(f"FP32 {n}^3 implicit Smagorinsky")
        extra["les256_implicit_smagorinsky"], _ = leg(torch, capi, si, N, K, W, 152, kernel=step_kernel_name(n, n))
        si.close()
        del si
        torch.cuda.empty_cache()
        # the same LES on the D3Q15 lattice (Yu-type formula of the Section 5.4 route):
        # 15 x 4 B read + written + 8 B lagged s_nu = 128 B/node
        w = _workloads()
        p15 = w.params(w.load("C1"), lattice="D3Q15", grid={"nx": n, "ny": n, "nz": n})
        s15 = lbm.LBM(p15, lbm.rho_u_field(np.zeros((n, n, n)), u))
        log(f"D3Q15 FP32 {n}^3 LES")
        extra["les256_d3q15"], _ = leg(torch, capi, s15, N, K, W, 128)
        s15.close()
        del s15
        torch.cuda.empty_cache()
        extra["channel_powerlaw"] = channel_runs(torch, capi, lbm, K, W)
        extra["strain_formulas_256"] = strain_formulas(torch, np, capi, lbm, u, 50, kernel_source_sha(STRAIN_SOURCES))
        extra["adjoint_c4"] = adjoint_run(torch, np, synth, capi, lbm, W)
        torch.cuda.empty_cache()
        extra["adjoint_c4_smagorinsky"] = adjoint_run(torch, np, synth, capi, lbm, W, visc="smagorinsky")
        extra["other_kernels"] = other_kernels(torch, np, synth, capi, lbm, u, 20, K, W)
        cp = copy_bandwidth(torch, capi)
        extra.update(cp)
        extra["step_over_stream_copy"] = round(result["roofline"]["achieved"] / cp["stream_copy_GBps"], 4)
        result["extra"] = extra

    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on one thread")
        result["cpu_baseline"] = cpu_baseline(u)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
