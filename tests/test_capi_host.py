"""Host-only checks of the C ABI: the library loads, exports every entry point that
include/lbm.h declares, and validates arguments before touching the GPU."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def _declared():
    text = (ROOT / "include" / "lbm.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("lbm_init", "lbm_step", "lbm_strain", "lbm_adjoint_step", "lbm_reduce", "lbm_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1704_07559_amd import capi
    lib = ctypes.CDLL(capi.library_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(capi.EXPORTED) == set(_declared())
    # the ctypes mirror of lbm_params has the library's layout
    assert capi._lib.lbm_params_size() == ctypes.sizeof(capi.lbm_params)


def test_population_bytes_and_validation():
    from paper_1704_07559_amd import capi
    s = [0.0, 1.19, 1.4, 0.0, 1.2, 0.0, 1.2, 0.0, 1.2, 1.25, 1.4, 1.25, 1.4, 1.25, 1.25, 1.25, 1.98, 1.98, 1.98]
    p = capi.Params(nx=32, ny=16, nz=8, s=s)
    assert capi.lbm_population_bytes(p) == 19 * 32 * 16 * 8 * 4
    p.storage = capi.LBM_F16
    assert capi.lbm_population_bytes(p) == 19 * 32 * 16 * 8 * 2
    bad = capi.Params(nx=0, ny=16, nz=8, s=s)
    assert capi.lbm_population_bytes(bad) == 0
    assert capi.lbm_population_bytes(capi.Params(nx=32, ny=16, nz=8, s=s, strain_force_correction=1)) > 0
    assert capi.lbm_population_bytes(capi.Params(nx=32, ny=16, nz=8, s=s, strain_force_correction=2)) == 0
    uneq = list(s)
    uneq[13] = 1.3
    assert capi.lbm_population_bytes(capi.Params(nx=4, ny=4, nz=4, s=uneq)) == 0
    assert capi.lbm_population_bytes(capi.Params(nx=4, ny=4, nz=2, lattice=capi.LBM_D2Q9, s=s)) == 0


def test_size_limits_and_other_lattices():
    """32-bit plane offsets: N must stay below 2^30 nodes; D3Q15 sizing and its s_nu slots;
    the implicit coupling only on D3Q19."""
    from paper_1704_07559_amd import capi
    s = [0.0, 1.19, 1.4, 0.0, 1.2, 0.0, 1.2, 0.0, 1.2, 1.25, 1.4, 1.25, 1.4, 1.25, 1.25, 1.25, 1.98, 1.98, 1.98]
    assert capi.lbm_population_bytes(capi.Params(nx=1024, ny=1024, nz=1023, s=s)) == 19 * 4 * 1024 * 1024 * 1023
    assert capi.lbm_population_bytes(capi.Params(nx=1024, ny=1024, nz=1024, s=s)) == 0
    assert capi.lbm_population_bytes(capi.Params(nx=1, ny=1, nz=1, s=s)) == 19 * 4
    # one z-plane of the row-interleaved buffer (ny * 19 * nx elements) must stay below 4 GiB
    assert capi.lbm_population_bytes(capi.Params(nx=8192, ny=8192, nz=1, s=s)) == 0
    assert capi.lbm_population_bytes(capi.Params(nx=8192, ny=8192, nz=1, s=s, storage=capi.LBM_F16)) == \
        19 * 2 * 8192 * 8192
    s15 = [0.0, 1.6, 1.2, 0.0, 1.6, 0.0, 1.6, 0.0, 1.6, 1.25, 1.25, 1.25, 1.25, 1.25, 1.2] + [0.0] * 4
    assert capi.lbm_population_bytes(capi.Params(nx=6, ny=5, nz=4, lattice=capi.LBM_D3Q15, s=s15)) == 15 * 4 * 120
    uneq = list(s15)
    uneq[12] = 1.3
    assert capi.lbm_population_bytes(capi.Params(nx=6, ny=5, nz=4, lattice=capi.LBM_D3Q15, s=uneq)) == 0
    imp = capi.LBM_VISC_SMAGORINSKY_IMPLICIT
    assert capi.lbm_population_bytes(capi.Params(nx=6, ny=5, nz=4, lattice=capi.LBM_D3Q15, s=s15,
                                                 visc_kind=imp)) == 15 * 4 * 120
    s9 = [0.0, 1.6, 1.2, 0.0, 1.6, 0.0, 1.6, 1.25, 1.25] + [0.0] * 10
    assert capi.lbm_population_bytes(capi.Params(nx=6, ny=5, nz=1, lattice=capi.LBM_D2Q9, s=s9,
                                                 visc_kind=imp)) == 9 * 4 * 30
    assert capi.lbm_population_bytes(capi.Params(nx=6, ny=5, nz=4, s=s, visc_kind=imp)) == 19 * 4 * 120
    assert capi.lbm_population_bytes(capi.Params(nx=6, ny=5, nz=4, lattice=7, s=s)) == 0


def test_largest_boxes_sit_at_the_limit():
    """The boxes of the maximum-size GPU tests are accepted, and one more row in y is not."""
    from paper_1704_07559_amd import capi
    from tests.test_gpu_maxsize import BOXES, _spec
    for name, (q, storage, shape) in BOXES.items():
        _, cp = _spec(q, shape, storage)
        elem = 4 if storage == "f32" else 2
        assert shape[1] * q * shape[2] * elem < 2 ** 32 <= (shape[1] + 1) * q * shape[2] * elem, name
        assert capi.lbm_population_bytes(cp) == q * elem * shape[0] * shape[1] * shape[2], name
        cp.ny += 1
        assert capi.lbm_population_bytes(cp) == 0, name


def test_init_rejects_bad_arguments_without_a_gpu():
    """Every case here fails validation, which runs before any HIP call or launch."""
    from paper_1704_07559_amd import capi
    s = [0.0, 1.19, 1.4, 0.0, 1.2, 0.0, 1.2, 0.0, 1.2, 1.25, 1.4, 1.25, 1.4, 1.25, 1.25, 1.25, 1.98, 1.98, 1.98]
    p = capi.Params(nx=8, ny=8, nz=8, s=s)
    nbytes = capi.lbm_population_bytes(p)
    cases = [
        (p, 1 << 20, 1 << 20, None),                     # aliased buffers
        (p, 1 << 20, (1 << 20) + nbytes // 2, None),     # overlapping buffers
        (p, (1 << 20) + 4, 1 << 24, None),               # misaligned buffer
        (p, None, 1 << 24, None),                        # missing buffer
        (capi.Params(nx=8, ny=8, nz=8, s=s, visc_kind=capi.LBM_VISC_SMAGORINSKY), 1 << 20, 1 << 24, None),
        (capi.Params(nx=8, ny=8, nz=8, s=s, visc_kind=capi.LBM_VISC_POWERLAW, K_pl=-1.0), 1 << 20, 1 << 24, 1 << 28),
        (capi.Params(nx=8, ny=1, nz=8, s=s, walls_y=1), 1 << 20, 1 << 24, None),
    ]
    for params, a, b, snu in cases:
        with pytest.raises(capi.LBMError) as e:
            capi.lbm_init(params, a, b, snu, None, None, stream=0)
        assert e.value.status == capi.LBM_EINVAL, capi.lbm_last_error()


def test_stream_copy_rejects_bad_arguments_without_a_gpu():
    """Validation of the copy runs before any HIP call (no launch happens here)."""
    from paper_1704_07559_amd import capi
    for src, dst, n in ((None, 1 << 24, 64), (1 << 20, None, 64), ((1 << 20) + 8, 1 << 24, 64),
                        (1 << 20, (1 << 24) + 4, 64), (1 << 20, 1 << 24, 40), (1 << 20, (1 << 20) + 32, 64),
                        ((1 << 20) + 32, 1 << 20, 64)):
        with pytest.raises(capi.LBMError) as e:
            capi.lbm_stream_copy(src, dst, n, stream=0)
        assert e.value.status == capi.LBM_EINVAL, (src, dst, n)


def test_reduce_async_rejects_bad_arguments_without_a_gpu():
    from paper_1704_07559_amd import capi
    for ctx, out in ((None, 1 << 20), (1 << 12, None), (1 << 12, (1 << 20) + 4)):
        st = capi._lib.lbm_reduce_async(ctx, out, None)
        assert st == capi.LBM_EINVAL, (ctx, out, st)


def test_status_strings():
    from paper_1704_07559_amd import capi
    assert capi.lbm_status_string(capi.LBM_OK) == "LBM_OK"
    assert "invalid" in capi.lbm_status_string(capi.LBM_EINVAL)
