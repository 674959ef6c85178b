"""Host-side pieces of the benchmark: the algorithmic byte counts it divides
by the measured times, the counter guard, and the multi-GPU refusal."""
import json
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402
import workloads as W  # noqa: E402


@pytest.mark.parametrize("name,floor", [
    # N (8d + 4) + G (8 + 8F): positions in and out, ids, the field read and
    # written, each deposited field written once and read once
    (W.PERIODIC_1K, 1000 * 20 + 64 ** 2 * 16),
    (W.WALLS_100K, 100000 * 20 + 512 ** 2 * 24),
    (W.BLOBS_1M, 1000000 * 28 + 128 ** 3 * 16),
    (W.ADJOINT_50K, 50000 * 20 + 256 ** 2 * 24),
])
def test_floor_bytes(name, floor):
    assert bench.floor_bytes(W.workload(name)) == floor


def test_floor_of_the_3d_run_is_61_6_MB():
    assert abs(bench.floor_bytes(W.workload(W.BLOBS_1M)) / 1e6 - 61.55) < 0.01


def test_stage_bytes_of_the_3d_run():
    w = W.workload(W.BLOBS_1M)
    N, G = 1000000, 128 ** 3
    assert bench.algorithmic_bytes("update", w, 1) == N * 28 + 4 * G
    assert bench.algorithmic_bytes("deposit", w, 1) == N * 13 + 4 * G
    assert bench.algorithmic_bytes("pde", w, 1) == G * 12
    assert bench.algorithmic_bytes("scatter", w, 1) == N * 32


def test_counter_guard_follows_the_sources_and_the_workload():
    assert bench.counters_valid("3d_periodic_1M_blobs") == (
        bench.sources_sha() == bench.COUNTER_SOURCES_SHA)
    assert not bench.counters_valid("2d_walls_100k")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
