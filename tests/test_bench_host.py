"""Host-side checks of bench.py (no GPU): the one-GPU contract, the traffic and VALU record lookups,
the relaxation-rate tables."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record_matches_only_its_kernel_source(tmp_path, monkeypatch):
    sha = bench.kernel_source_sha()
    assert len(sha) == 16
    rec = bench.read_traffic("step_d3q19_f32_les256", sha)
    assert rec is None or 150 * 256**3 < rec < 175 * 256**3      # bytes per launch, near 160 B/node
    assert bench.read_traffic("step_d3q19_f32_les256", "0" * 16) is None
    assert bench.read_traffic("no_such_kernel", sha) is None


def test_rate_tables():
    r19, r15 = bench.rates(0.5 + 1.0 / 3.0), bench.rates15(0.8)
    assert len(r19) == 19 and len(r15) == 15
    assert {r19[k] for k in (9, 11, 13, 14, 15)} == {1.0 / (0.5 + 1.0 / 3.0)}
    assert {r15[k] for k in range(9, 14)} == {1.0 / 0.8}
    assert r19[0] == r19[3] == r19[5] == r19[7] == 0.0 and r15[0] == r15[3] == r15[5] == r15[7] == 0.0


def test_valu_record_matches_only_its_kernel_source():
    sha = bench.kernel_source_sha()
    v = bench.read_valu("f16_les384", sha)
    # one wave per 64 nodes, a few hundred VALU instructions per wave
    assert v is None or 100 * 384**3 / 64 < v < 1000 * 384**3 / 64
    assert bench.read_valu("f16_les384", "0" * 16) is None
    assert bench.read_valu("no_such_run", sha) is None
    assert bench.valu_frac(None, 1e-3) is None
    # the issue ceiling: 614.4e9 wave instructions per second
    assert abs(bench.valu_frac(614.4e6, 1e-3) - 1.0) < 1e-9


def test_step_kernel_name_follows_the_launch_rule():
    """The instance named in the roofline record: whole 256-node rows exchange through LDS
    (pull mode 2), 384-node rows split into 128-node segments (mode 0), rows of 32 nodes are
    covered by one masked block (mode 1), the 128-wide channel with walls is mode 2."""
    assert bench.step_kernel_name(256, 256) == "lbm::d3q19::step_kernel<float, false, 2, false>"
    assert bench.step_kernel_name(384, 384, "f16") == "lbm::d3q19::step_kernel<_Float16, false, 0, false>"
    assert bench.step_kernel_name(384, 384, "bf16") == "lbm::d3q19::step_kernel<__bf16, false, 0, false>"
    assert bench.step_kernel_name(32, 32) == "lbm::d3q19::step_kernel<float, false, 1, false>"
    assert bench.step_kernel_name(128, 128, walls=True) == "lbm::d3q19::step_kernel<float, true, 2, false>"
    assert bench.step_kernel_name(64, 6) == "lbm::d3q19::step_kernel<float, false, 1, false>"  # 4 rows do not tile 6


def test_strain_valu_record_matches_only_its_kernel_sources():
    v = bench.read_valu_strain(bench.kernel_source_sha(bench.STRAIN_SOURCES))
    assert v is None or (v["query_chai"] > v["query_yu"] and v["step_drive_chai"] > v["step_drive_yu"])
    assert bench.read_valu_strain("0" * 16) is None


def test_resource_remarks_are_parsed():
    """The kernel-resource-usage remarks hipcc prints are turned into one record per kernel."""
    from paper_1704_07559_amd.build import parse_resource_remarks
    text = "\n".join([
        "k.hip:1:1: remark: Function Name: _Z1kv [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:1:1: remark:     VGPRs: 80 [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:1:1: remark:     Occupancy [waves/SIMD]: 6 [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:1:1: remark:     Dynamic Stack: False [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:1:1: remark:     LDS Size [bytes/block]: 10240 [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:2:1: remark: Function Name: _Z1jv [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:2:1: remark:     VGPRs: 90 [-Rpass-analysis=kernel-resource-usage]",
    ])
    ks = parse_resource_remarks(text, "k.hip")
    assert ks == [{"file": "k.hip", "kernel": "_Z1kv", "vgprs": 80, "scratch": 0, "waves_per_simd": 6, "lds": 10240},
                  {"file": "k.hip", "kernel": "_Z1jv", "vgprs": 90}]
