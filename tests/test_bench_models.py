"""The benchmark's byte models and counter bookkeeping (CPU only).

B_alg per nonzero per mode follows the paper's traffic model (Sec. V, impact
of rank): record read + remap write + the N-1 gathered factor rows; the
output rows are added per mode.  Per-nonzero figures for the five
workloads, worked out by hand: 288 / 160 B (3 modes, R 32, FP32 / BF16),
424 / 232 B (4 modes, R 32), 304 / 176 B (5 modes, R 16).
"""
import pytest

import bench


@pytest.mark.parametrize("N,R,fp32,bf16", [(3, 32, 288, 160), (4, 32, 424, 232),
                                           (5, 16, 304, 176), (3, 16, 160, 96)])
def test_per_nonzero_bytes(N, R, fp32, bf16):
    dims = (10,) * N
    nnz = 1000
    out = 10 * R * 4
    assert bench.b_alg_mode(dims, nnz, R, 0, 4) == nnz * fp32 + out
    assert bench.b_alg_mode(dims, nnz, R, 0, 2) == nnz * bf16 + out


def test_workload2_sweep_bytes():
    dims, nnz, R = (50000, 40000, 30000), 20_000_000, 32
    sweep = sum(bench.b_alg_mode(dims, nnz, R, n, 4) for n in range(3))
    assert sweep == 3 * nnz * 288 + sum(dims) * R * 4
    assert abs(sweep / 1e9 - 17.3) < 0.05
    # kernel split: MTTKRP launch = record + gathers + output; remap = 2E + 4
    k = bench.b_alg_mttkrp_kernel(dims, nnz, R, 0, 4)
    assert k == nnz * (16 + 2 * 32 * 4) + dims[0] * R * 4
    assert bench.b_alg_remap_kernel(dims, nnz) == nnz * 36
    # stored records of 12 bytes (16 + 16 + 15 coordinate bits in two words)
    assert bench.b_alg_remap_kernel(dims, nnz, 12) == nnz * 28
    # compulsory: records once, each input factor once, the output
    m = bench.b_min_mttkrp_kernel(dims, nnz, R, 0, 4)
    assert m == nnz * 16 + (40000 + 30000) * R * 4 + 50000 * R * 4
    assert bench.b_min_mttkrp_kernel(dims, nnz, R, 0, 4, 12) == m - nnz * 4


def test_counter_summary_is_used_only_for_the_profiled_sources(tmp_path):
    sha = bench.source_sha()
    good = tmp_path / "good.txt"
    good.write_text(f"# header: x\nfetch_bytes_per_launch: 123\nsource_sha: {sha}\n")
    assert bench.counter_traffic(str(good), "fetch_bytes_per_launch") == 123
    stale = tmp_path / "stale.txt"
    stale.write_text("fetch_bytes_per_launch: 123\nsource_sha: 0000000000000000\n")
    assert bench.counter_traffic(str(stale), "fetch_bytes_per_launch") is None
    assert bench.counter_traffic(str(tmp_path / "missing.txt"), "x") is None
    assert bench.counter_traffic(str(good), "write_bytes_per_launch") is None

