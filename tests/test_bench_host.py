"""Host-side checks of the benchmark script: the committed HBM byte records and
the roofline arithmetic (no GPU work)."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

VOXELS = {22: 256 ** 3, 32: 256 ** 3, 64: 16 * 128 ** 3, None: 256 ** 3}
ALGO_BYTES = {1: bench.BYTES_PER_VOXEL_STEP, 0: bench.BYTES_PER_VOXEL_GRAD, 2: bench.BYTES_PER_VOXEL_ADAM}


def _records():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        return json.load(fh)


def test_traffic_records_are_consistent_with_their_counters():
    t = _records()
    assert t["fetch_scale"] == 2.0 and t["write_scale"] == 1.0
    assert len(t["kernel_sources_sha256_prefix"]) == 16
    seen = set()
    for r in t["records"]:
        key = (r["kernel"], r["z_chunk"])
        assert key not in seen
        seen.add(key)
        scaled = (r["fetch_kib_raw"] * t["fetch_scale"] + r["write_kib_raw"] * t["write_scale"]) * 1024
        assert abs(scaled - r["traffic_bytes"]) <= 1024
        # every counted byte total lies at or just above the kernel's algorithmic bytes
        if r["kernel"].startswith("energy_sweep_cols"):
            algo = bench.BYTES_PER_VOXEL_ENERGY * VOXELS[None]
        else:
            mode = int(r["kernel"].split(",")[4])
            algo = ALGO_BYTES[mode] * VOXELS[r["z_chunk"]]
        assert 1.0 <= r["traffic_bytes"] / algo <= 1.15, r


def test_measured_traffic_matches_kernel_and_launch():
    t = _records()
    r = t["records"][0]
    if t["kernel_sources_sha256_prefix"] != bench.kernel_hash():
        assert bench.measured_traffic(r["kernel"], r["z_chunk"]) is None
    else:
        assert bench.measured_traffic(r["kernel"], r["z_chunk"]) == r["traffic_bytes"]
    assert bench.measured_traffic(r["kernel"], -1) is None
    assert bench.measured_traffic("no_such_kernel", r["z_chunk"]) is None


def test_roofline_picks_the_binding_roof():
    # 230 operations and 8 bytes per voxel at 256^3 in 86 us: ALU-bound
    roof, other = bench.roofline(230, 8, 256 ** 3, 86.0, "k", None)
    assert roof["bound"] == "alu" and other["bound"] == "hbm"
    assert roof["achieved"] == pytest.approx(230 * 256 ** 3 / 86e-6 / 1e12)
    assert roof["frac"] == pytest.approx(roof["achieved"] / bench.FP32_VECTOR_PEAK_TFLOPS)
    assert roof["frac_of_unpacked_peak"] == pytest.approx(2 * roof["frac"])
    assert other["achieved"] == pytest.approx(8 * 256 ** 3 / 86e-6 / 1e9)
    # 4 bytes and 1 operation per voxel: HBM-bound
    roof, _ = bench.roofline(1, 4, 256 ** 3, 10.0, "k", 123)
    assert roof["bound"] == "hbm" and roof["traffic"] == 123 and "frac_of_unpacked_peak" not in roof


def test_flop_counts_drop_the_s_terms_for_symmetric_p():
    assert bench.flops_per_voxel(bench.HELFRICH_SC) == bench.FLOPS_PER_VOXEL - bench.FLOPS_S_TERMS
    assert bench.flops_per_voxel((1.0, 0.0, 2.0, 0.0, 0.0, 0.0)) == bench.FLOPS_PER_VOXEL
    assert bench.forward_flops_per_voxel(bench.HELFRICH_SC) == 97 - 18


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr
