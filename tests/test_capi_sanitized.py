"""The C ABI's host code under the address and undefined-behaviour sanitizers (no GPU).

The library's host layer (argument validation, the context, the error strings) is rebuilt
with -fsanitize=address,undefined and loaded into a fresh Python with the sanitizer runtime
preloaded; every entry point is driven through its validation paths (invalid parameters,
NULL, misaligned, aliased and overlapping buffers, size limits, unsupported combinations) and
through lbm_init's clean-up after its first HIP call fails on a machine without a GPU. Any
sanitizer report aborts the child, so the test passes only on a clean run."""
import os
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]

CHILD = r'''
import ctypes, sys
sys.path.insert(0, sys.argv[1])
from paper_1704_07559_amd import capi
lib = capi._lib
s = [0.0, 1.19, 1.4, 0.0, 1.2, 0.0, 1.2, 0.0, 1.2, 1.25, 1.4, 1.25, 1.4, 1.25, 1.25, 1.25, 1.98, 1.98, 1.98]
ok = capi.Params(nx=8, ny=8, nz=8, s=s)
n_checked = 0
def expect(status, want, what):
    global n_checked
    assert status == want, (what, status, capi.lbm_last_error())
    assert isinstance(lib.lbm_last_error(), bytes)
    n_checked += 1
assert capi.lbm_population_bytes(ok) == 19 * 512 * 4
for bad in (capi.Params(nx=0, ny=8, nz=8, s=s), capi.Params(nx=8, ny=8, nz=8, s=s, lattice=7),
            capi.Params(nx=8, ny=8, nz=8, s=s, storage=9), capi.Params(nx=4, ny=4, nz=2, lattice=capi.LBM_D2Q9, s=s),
            capi.Params(nx=1024, ny=1024, nz=1024, s=s), capi.Params(nx=8, ny=8, nz=8, s=s, rho0=-1.0),
            capi.Params(nx=8, ny=8, nz=8, s=s, visc_kind=9), capi.Params(nx=8, ny=1, nz=8, s=s, walls_y=1),
            capi.Params(nx=8, ny=8, nz=8, s=s, strain_force_correction=3),
            capi.Params(nx=8, ny=8, nz=8, s=s, force=(float("nan"), 0.0, 0.0))):
    assert capi.lbm_population_bytes(bad) == 0
    n_checked += 1
assert lib.lbm_population_bytes(None) == 0
nb = capi.lbm_population_bytes(ok)
out = ctypes.c_void_p()
P = ok.to_c()
for a, b, snu in ((1 << 20, 1 << 20, None), (1 << 20, (1 << 20) + nb // 2, None), ((1 << 20) + 4, 1 << 24, None),
                  (None, 1 << 24, None)):
    expect(lib.lbm_init(ctypes.byref(out), ctypes.byref(P), a, b, snu, None, None, None), capi.LBM_EINVAL, "init")
    assert out.value is None
expect(lib.lbm_init(None, ctypes.byref(P), 1 << 20, 1 << 24, None, None, None, None), capi.LBM_EINVAL, "init out")
Ps = capi.Params(nx=8, ny=8, nz=8, s=s, visc_kind=capi.LBM_VISC_SMAGORINSKY).to_c()
expect(lib.lbm_init(ctypes.byref(out), ctypes.byref(Ps), 1 << 20, 1 << 24, None, None, None, None), capi.LBM_EINVAL,
       "init without s_nu field")
# valid arguments: validation passes, the first HIP call fails without a GPU, and the
# half-built context is freed
st = lib.lbm_init(ctypes.byref(out), ctypes.byref(P), 1 << 20, 1 << 24, None, None, None, None)
assert st != capi.LBM_OK and out.value is None, st
n_checked += 1
for fn, args in (("lbm_step", (None, 1, None, 1, None, None)), ("lbm_strain", (None, 1, 1 << 20, None)),
                 ("lbm_reduce", (None, None, None)), ("lbm_reduce_async", (None, 1 << 20, None)),
                 ("lbm_get_populations", (None, 1 << 20, None)), ("lbm_set_populations", (None, 1 << 20, None)),
                 ("lbm_save_state", (None, 1 << 20, None)), ("lbm_load_state", (None, 1 << 20, None)),
                 ("lbm_set_step_count", (None, 3)),
                 ("lbm_adjoint_step", (None, 1 << 20, 1 << 21, 1 << 22, None, None)),
                 ("lbm_adjoint_steps", (None, 2, 1 << 20, 1 << 21, 1 << 22, None, None)),
                 ("lbm_adjoint_steps_noalloc", (None, 2, 1 << 20, 1 << 21, None, None)),
                 ("lbm_strain_loss_seed", (None, 1 << 20, None, None, None)),
                 ("lbm_init_adjoint", (None, 1 << 20, 1 << 21, 1 << 22, None))):
    expect(getattr(lib, fn)(*args), capi.LBM_EINVAL, fn)
for src, dst, n in ((None, 1 << 24, 64), ((1 << 20) + 8, 1 << 24, 64), (1 << 20, 1 << 24, 40),
                    (1 << 20, (1 << 20) + 32, 64)):
    expect(lib.lbm_stream_copy(src, dst, n, None), capi.LBM_EINVAL, "copy")
assert lib.lbm_step_count(None) == -1 and lib.lbm_state_bytes(None) == 0
assert lib.lbm_save_planes(None) == 0 and lib.lbm_adjoint_planes(None) == 0
lib.lbm_destroy(None)
for code in range(-8, 2):
    assert isinstance(lib.lbm_status_string(code), bytes)
print("checked", n_checked)
'''


@pytest.mark.slow
def test_host_layer_is_clean_under_asan_and_ubsan(tmp_path):
    from paper_1704_07559_amd import build
    lib = build.build_sanitized(tmp_path / "liblbm_sanitized.so")
    runtime = build.sanitizer_runtime()
    assert Path(runtime).exists(), runtime
    env = dict(os.environ, LD_PRELOAD=runtime, LBM_LIBRARY=str(lib),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", CHILD, str(ROOT)], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-6000:])
    assert "checked" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
