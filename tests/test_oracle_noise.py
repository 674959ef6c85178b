"""Pins of the oracle's noise: Philox4x32-10 words, uniforms and normals.

The paper draws xi ~ N(0, I) per agent and step (eq. sde_EM).  The oracle's
generator is Philox4x32-10 (Salmon et al., SC'11).  Its words are pinned to
an independent implementation (rocRAND's engine, compiled and run on the
host); its normals are pinned statistically.
"""
import shutil
import subprocess
from pathlib import Path

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads as W

PIN = Path(__file__).parent / "pins" / "rocrand_philox.cpp"


def _rocrand_binary(tmp_path_factory):
    cxx = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not Path(cxx).exists():
        pytest.skip("no HIP compiler to build the rocRAND pin")
    out = tmp_path_factory.mktemp("pin") / "rocrand_philox"
    subprocess.run([cxx, "-O1", "-x", "hip", "--offload-arch=gfx950", str(PIN), "-o", str(out)],
                   check=True, capture_output=True)
    return out


@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    return _rocrand_binary(tmp_path_factory)


def test_philox_matches_rocrand(rocrand_pin, oracle_lib):
    rng = np.random.default_rng(7)
    ctr = rng.integers(0, 2**32, size=(400, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(400, 2), dtype=np.uint64).astype(np.uint32)
    # edge counters / keys: all zero, all ones, the step/id/inst layout
    ctr[0] = 0; key[0] = 0
    ctr[1] = 0xFFFFFFFF; key[1] = 0xFFFFFFFF
    ctr[2] = [199, 999_999, 0, 0]; key[2] = [1003, 0]
    ctr[3] = [5, 17, 255, 0]; key[3] = [0xDEADBEEF, 0x12345678 ^ 255]
    text = "\n".join(" ".join("%08x" % v for v in (*c, *k)) for c, k in zip(ctr, key)) + "\n"
    res = subprocess.run([str(rocrand_pin)], input=text, capture_output=True, text=True, check=True)
    ref = np.array([[int(t, 16) for t in line.split()] for line in res.stdout.strip().splitlines()],
                   dtype=np.uint32)
    got = oracle.philox(ctr, key)
    assert ref.shape == got.shape
    assert np.array_equal(ref, got)


def test_uniform_mapping_range_and_lattice(oracle_lib):
    # The normals of id i at step s come from one Philox block; their uniforms
    # are odd multiples of 2^-24 in (0, 1): check via the inverse Box-Muller
    # radius of the first pair, which must be one of those lattice values.
    w = W.workload(W.PERIODIC_1K)
    p = oracle.params(w)
    ids = np.arange(20000, dtype=np.uint32)
    xi = oracle.normals(p, 3, ids)
    u0 = np.exp(-0.5 * (xi[:, 0] ** 2 + xi[:, 1] ** 2))
    q = u0 * 2**24
    assert np.all(np.abs(q - np.rint(q)) < 1e-6 * q + 1e-9)
    qi = np.rint(q).astype(np.int64)
    assert np.all(qi % 2 == 1) and qi.min() >= 1 and qi.max() <= 2**24 - 1
    # and the same block words give the same value through philox()
    ctr = np.stack([np.full(len(ids), 3), ids, np.zeros(len(ids)), np.zeros(len(ids))], 1)
    key = np.stack([np.full(len(ids), p.seed & 0xFFFFFFFF), np.full(len(ids), p.seed >> 32)], 1)
    words = oracle.philox(ctr, key)
    assert np.array_equal(((words[:, 0] >> 8) | 1).astype(np.int64), qi)


@pytest.mark.parametrize("dim", [2, 3])
def test_normals_are_standard(dim, oracle_lib):
    w = W.scaled(W.workload(W.BLOBS_1M if dim == 3 else W.PERIODIC_1K), n_agents=10)
    p = oracle.params(w)
    ids = np.arange(400_000, dtype=np.uint32)
    xi = np.concatenate([oracle.normals(p, s, ids) for s in (0, 1)], 0)
    n = len(xi)
    for a in range(dim):
        col = xi[:, a]
        assert abs(col.mean()) < 5 / np.sqrt(n)
        assert abs(col.var() - 1) < 5 * np.sqrt(2 / n)
        assert stats.kstest(col, "norm").pvalue > 1e-3
    # components, steps and ids are uncorrelated
    c = np.corrcoef(xi.T)
    assert np.all(np.abs(c - np.eye(dim)) < 5 / np.sqrt(n))
    a0 = oracle.normals(p, 0, ids)[:, 0]
    a1 = oracle.normals(p, 1, ids)[:, 0]
    assert abs(np.corrcoef(a0, a1)[0, 1]) < 5 / np.sqrt(len(a0))
    assert abs(np.corrcoef(a0[:-1], a0[1:])[0, 1]) < 5 / np.sqrt(len(a0))


def test_instances_draw_different_streams(oracle_lib):
    w = W.workload(W.ENSEMBLE_256)
    ids = np.arange(5000, dtype=np.uint32)
    x0 = oracle.normals(oracle.params(w, 0), 0, ids)
    x1 = oracle.normals(oracle.params(w, 1), 0, ids)
    assert abs(np.corrcoef(x0[:, 0], x1[:, 0])[0, 1]) < 5 / np.sqrt(len(ids))
