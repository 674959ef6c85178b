"""Pins of the oracle's neighbour sets and pair forces.

* Neighbour sets: against scipy's KD-tree (periodic `boxsize` for the torus),
  an implementation that shares nothing with the oracle; and all-pairs vs
  cell-list enumeration.
* Forces: two-agent closed form |F| = k (d - r) along the line of centres,
  zero for r >= d and for coincident agents (the r > 0 guard of the
  interaction loop, Sect. 3.2), Newton's third law (sum F = 0) and bitwise
  antisymmetry of pair terms.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import workloads as W


def _pairs_kdtree(X, diam_of, L, periodic, cutoff):
    tree = cKDTree(X, boxsize=L if periodic else None)
    pairs = tree.query_pairs(cutoff, output_type="ndarray")
    return pairs


@pytest.mark.parametrize("name,n", [(W.PERIODIC_1K, 3000), (W.WALLS_100K, 6000),
                                    (W.BLOBS_1M, 6000), (W.ADJOINT_50K, 4000)])
def test_neighbour_sets_vs_kdtree(name, n, oracle_lib):
    w = W.scaled(W.workload(name), n_agents=n)
    if name == W.BLOBS_1M:
        # blobs shrunk so that 6000 agents still have many contacts
        w = W.scaled(w, n_agents=n)
    inp = W.make_inputs(w)
    X32, sp = inp["x0"], inp["species0"]
    if name == W.BLOBS_1M:
        X32 = np.mod(X32 * np.float32(0.2), np.float32(1.0)).astype(np.float32)
    ids = np.arange(n, dtype=np.uint32)
    diam = [s.diameter for s in w.species]
    cnt_b, h_b = oracle.neighbours_f32(w.dim, w.periodic, w.L, X32, sp, ids, diam, mode=0)
    cnt_c, h_c = oracle.neighbours_f32(w.dim, w.periodic, w.L, X32, sp, ids, diam, mode=1)
    assert np.array_equal(cnt_b, cnt_c) and np.array_equal(h_b, h_c)
    assert cnt_b.sum() > n // 10
    # scipy: float64 distances of the same float32 coordinates
    X = X32.astype(np.float64)
    dmax = max(diam)
    pairs = _pairs_kdtree(X, diam, w.L, w.periodic, dmax)
    i, j = pairs[:, 0], pairs[:, 1]
    dx = X[j] - X[i]
    if w.periodic:
        dx -= w.L * np.rint(dx / w.L)
    r = np.sqrt((dx * dx).sum(1))
    dij = 0.5 * (np.asarray(diam)[sp[i]] + np.asarray(diam)[sp[j]])
    keep = r < dij
    # pairs within float32 rounding of the contact distance may be decided
    # either way; everything else must agree exactly
    edge = np.abs(r - dij) < 1e-6 * dij
    ref = np.zeros(n, np.int64)
    np.add.at(ref, i[keep], 1)
    np.add.at(ref, j[keep], 1)
    amb = np.zeros(n, np.int64)
    np.add.at(amb, i[edge], 1)
    np.add.at(amb, j[edge], 1)
    diff = np.abs(ref - cnt_b.astype(np.int64))
    assert np.all(diff <= amb)
    sure = amb == 0
    hs = np.zeros(n, np.uint64)
    hid = np.array([oracle.hash_id(k) for k in range(n)], np.uint64)
    with np.errstate(over="ignore"):
        np.add.at(hs, i[keep], hid[j[keep]])
        np.add.at(hs, j[keep], hid[i[keep]])
    assert np.array_equal(hs[sure], h_b[sure])


def _p(dim=2, periodic=True, k=100.0, diam=(0.01,), L=1.0, mode=0):
    w = W.Workload("t", dim, periodic, L, 16, 1e-5, k, 1.0, 0.0, 1,
                   tuple(W.Species(d, 1.0, 0.0, 0.0, 0.0) for d in diam),
                   (W.Instance(2, 1),))
    return oracle.params(w, mode=mode)


@pytest.mark.parametrize("dim", [2, 3])
def test_two_agent_force_closed_form(dim, oracle_lib):
    rng = np.random.default_rng(1)
    p = _p(dim=dim)
    for _ in range(50):
        r = rng.uniform(0.0005, 0.015)
        u = rng.standard_normal(dim)
        u /= np.linalg.norm(u)
        a = rng.uniform(0.2, 0.8, dim)
        X = np.stack([a, a + r * u])
        F = oracle.forces(p, X, np.zeros(2, np.uint8))
        mag = p.k * max(0.01 - r, 0.0)
        np.testing.assert_allclose(F[0], -mag * u, rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(F[1], mag * u, rtol=1e-9, atol=1e-13)


def test_force_across_periodic_seam_and_walls(oracle_lib):
    p = _p(dim=2, periodic=True)
    X = np.array([[0.001, 0.5], [0.997, 0.5]])  # 0.004 apart through x = 0
    F = oracle.forces(p, X, np.zeros(2, np.uint8))
    np.testing.assert_allclose(F[0], [p.k * (0.01 - 0.004), 0.0], rtol=1e-9)
    np.testing.assert_allclose(F[1], [-p.k * (0.01 - 0.004), 0.0], rtol=1e-9)
    q = _p(dim=2, periodic=False)
    F = oracle.forces(q, X, np.zeros(2, np.uint8))
    assert np.all(F == 0.0)  # no seam with walls


def test_coincident_agents_no_force_and_contact_mean(oracle_lib):
    p = _p(dim=2, diam=(0.002, 0.004))
    X = np.array([[0.5, 0.5], [0.5, 0.5], [0.5029, 0.5]])
    sp = np.array([0, 0, 1], np.uint8)
    F = oracle.forces(p, X, sp)
    # agents 0 and 1 coincide: no force between them; agent 2 at 0.0029 from
    # both, contact distance (0.002 + 0.004) / 2 = 0.003
    mag = p.k * (0.003 - 0.0029)
    np.testing.assert_allclose(F[0], [-mag, 0], rtol=1e-9)
    np.testing.assert_allclose(F[1], [-mag, 0], rtol=1e-9)
    np.testing.assert_allclose(F[2], [2 * mag, 0], rtol=1e-9)


@pytest.mark.parametrize("name", [W.PERIODIC_1K, W.WALLS_100K, W.ADJOINT_50K])
def test_newton_third_law_and_modes(name, oracle_lib):
    w = W.scaled(W.workload(name), n_agents=3000)
    inp = W.make_inputs(w)
    X = inp["x0"].astype(np.float64) * (0.3 if name != W.WALLS_100K else 0.2)
    Fb = oracle.forces(oracle.params(w, mode=0), X, inp["species0"])
    Fc = oracle.forces(oracle.params(w, mode=1), X, inp["species0"])
    assert np.array_equal(Fb, Fc)
    tot = np.abs(Fb).sum()
    assert tot > 0
    assert np.all(np.abs(Fb.sum(0)) <= 1e-12 * tot)


def test_forces_subset_matches_full(oracle_lib):
    w = W.scaled(W.workload(W.BLOBS_1M), n_agents=5000)
    inp = W.make_inputs(w)
    X = inp["x0"].astype(np.float64) * 0.25
    p = oracle.params(w, mode=1)
    F = oracle.forces(p, X, inp["species0"])
    which = np.array([0, 17, 999, 4999])
    Fs = oracle.forces_subset(oracle.params(w, mode=0), X, inp["species0"], which)
    assert np.array_equal(F[which], Fs)
