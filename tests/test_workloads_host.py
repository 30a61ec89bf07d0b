"""The workload files (paper_1704_07559_amd/configs): each holds what its configuration
states, and the library parameters built from it carry those values (host only)."""
import pytest

from oracle import d2q9 as o9
from oracle import d3q15 as o15
from oracle import d3q19 as o19


@pytest.fixture(scope="module")
def w():
    from paper_1704_07559_amd import workloads
    return workloads


def test_every_workload_loads_and_builds(w):
    for name in ("C0", "C1", "C2", "C3", "C4"):
        cfg = w.load(name)
        assert cfg["name"] == name
        p = w.params(cfg)
        assert (p.nx, p.ny, p.nz) == (cfg["grid"]["nx"], cfg["grid"]["ny"], cfg["grid"]["nz"])


def test_headline_les(w):
    from paper_1704_07559_amd import capi
    cfg = w.load("C1")
    p = w.params(cfg)
    assert (p.nx, p.ny, p.nz, p.storage) == (256, 256, 256, capi.LBM_F32)
    assert p.visc_kind == capi.LBM_VISC_SMAGORINSKY and p.visc_strain == capi.LBM_STRAIN_YU
    assert p.c_smag == 0.1 and abs(p.nu0 - 1.0 / 300.0) < 1e-15 and cfg["steps"] == 1000
    assert cfg["init"] == {"kind": "spectrum", "seed": 1704, "u_rms": 0.04, "k0": 4.0, "delta_rho": 0.0}


def test_channel(w):
    from paper_1704_07559_amd import capi
    cfg = w.load("C2")
    assert cfg["viscosity"]["n_pl"] == [0.5, 1.0, 1.5] and cfg["steps"] == 5000
    for n in (0.5, 1.0, 1.5):
        p = w.params(cfg, n_pl=n)
        assert (p.nx, p.ny, p.nz, p.walls_y) == (128, 128, 512, 1) and tuple(p.force) == (0.0, 0.0, 1e-6)
        assert p.visc_kind == capi.LBM_VISC_POWERLAW and p.visc_strain == capi.LBM_STRAIN_CHAI
        # K = nu_ref * gamma_ref^(1 - n) with gamma_ref the Newtonian wall shear at nu_ref = 0.1
        gamma_ref = 1e-6 * 128 / (2 * 0.1)
        assert abs(p.K_pl - 0.1 * gamma_ref ** (1 - n)) < 1e-15 * p.K_pl and p.n_pl == n
    assert w.params(cfg, n_pl=1.0).K_pl == 0.1          # n = 1: the Newtonian viscosity itself
    with pytest.raises(ValueError):
        w.params(cfg, n_pl=0.7)


def test_half_storage_and_adjoint(w):
    from paper_1704_07559_amd import capi
    c3 = w.load("C3")
    assert [w.params(c3, storage=s).storage for s in ("f16", "bf16", "f32")] == [capi.LBM_F16, capi.LBM_BF16,
                                                                                 capi.LBM_F32]
    with pytest.raises(ValueError):
        w.params(w.load("C1"), storage="f16")            # C1 is FP32 only
    c4 = w.load("C4")
    p = w.params(c4)
    assert (p.nx, c4["steps"], c4["checkpoint_every"], p.visc_kind) == (128, 500, 50, capi.LBM_VISC_CONST)
    assert c4["force"] == {"kind": "uniform_random", "seed": 7559, "amplitude": 1e-6}


def test_rates_are_the_oracles_reading(w):
    """The non-viscous rates (reading R3 / R12 / R16) and s_nu = 1/tau_nu agree with the
    sets the oracles use, lattice by lattice."""
    for tau in (0.51, 0.8):
        assert w.rates_d3q19(tau) == pytest.approx(list(o19.default_rates(tau)), abs=0)
        assert w.rates_d3q15(tau) == pytest.approx(list(o15.default_rates(tau)), abs=0)
        assert w.rates_d2q9(tau) == pytest.approx(list(o9.default_rates(tau)), abs=0)
