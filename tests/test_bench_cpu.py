"""The benchmark's bookkeeping against the committed profile summaries (CPU
only): the kernel name it looks up is the one the kernel trace records, the
traffic and peak summaries parse, and the traffic figure belongs to the
current kernel sources."""
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def test_kernel_names_match_the_kernel_trace():
    with open(os.path.join(PROFILES, "k_tile_numeric_cube30_fp64.txt")) as f:
        text = f.read()
    # bench default on cube30: FP64, b = 13 (full K-steps), three directions,
    # 4 x 4 sub-tiles with four waves per sub-tile column
    fp64 = bench.kernel_name("tile", 0, 3, 3, 13)
    assert f"tc2::{fp64}(tc2::TileArgs)" in text
    assert fp64.endswith(", 4>")
    assert bench.kernel_name("tile", 3, 1, 0, 13).endswith(", 2>")          # D = 1, 8 x 8
    assert bench.kernel_name("tile", 1, 1, 0, 13).endswith(", 1>")          # plain FP32
    assert bench.kernel_name("tile", 3, 3, 3, 13).endswith(", 4>")          # FP32 with FP64 sums
    assert bench.kernel_name("tile", 3, 3, 3, 13, split=True).endswith("true, true, false, 4>")  # BF16 split
    assert bench.kernel_name("block", 0, 2, -1, 8) == "k_numeric<double, 2>"


def test_traffic_summary_belongs_to_the_current_sources():
    path = os.path.join(PROFILES, "k_tile_numeric_cube30_fp64_traffic.md")
    with open(path) as f:
        recorded = re.search(r"kernel_source_sha256_16: `([0-9a-f]{16})`", f.read()).group(1)
    traffic = bench.measured_traffic("k_tile_numeric", "cube30", "fp64")
    if recorded == bench.kernel_source_hash():
        assert traffic is not None and 1e11 < traffic < 1e14
    else:  # the kernels changed since the counters were taken: reported as unknown
        assert traffic is None


def test_trace_summary_records_the_same_source_hash_as_the_traffic_summary():
    with open(os.path.join(PROFILES, "k_tile_numeric_cube30_fp64.txt")) as f:
        trace = re.search(r"sha256\[:16\] = ([0-9a-f]{16})", f.read()).group(1)
    with open(os.path.join(PROFILES, "k_tile_numeric_cube30_fp64_traffic.md")) as f:
        traffic = re.search(r"kernel_source_sha256_16: `([0-9a-f]{16})`", f.read()).group(1)
    assert trace == traffic


def test_measured_peaks_parse():
    peaks = bench.measured_peaks()
    assert peaks is not None
    assert 0 < peaks["gemm_fp32_tflops"] <= bench.PEAK_TFLOPS["fp32"]
    assert 0 < peaks["gemm_fp64_tflops"] <= bench.PEAK_TFLOPS["fp64"]
    assert 0 < peaks["copy_GBps_read_plus_write"] <= bench.HBM_PEAK_GBS


def test_pack_units_keeps_order_and_bounds():
    from paper_2009_03551_amd import workloads as W

    class Sys:  # only the atom count matters for packing
        def __init__(self, nb):
            self.H = type("H", (), {"nb": nb})()

    sizes = [5, 7, 3, 20, 2, 2, 9]
    units = W.pack_units([Sys(n) for n in sizes], 12)
    assert [[s.H.nb for s in u] for u in units] == [[5, 7], [3], [20], [2, 2], [9]]
    assert all(sum(s.H.nb for s in u) <= 12 or len(u) == 1 for u in units)
    assert W.pack_units([], 12) == []
