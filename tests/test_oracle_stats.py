"""Pins of the oracle's ensemble statistics (the per-species histograms and
mean field of the experiment of Sect. 4, Fig. 1).

* numpy's histogramdd with edges linspace(0, L, m + 1) gives the same counts
  except for agents within float32 rounding of an edge (excluded);
* hand-placed agents land in the bin whose index is x-fastest;
* counts sum to the agent count, totals are the species counts, positions on
  the upper wall go to the last bin.
"""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("dim,m", [(2, 52), (3, 16), (2, 7)])
def test_species_hist_matches_histogramdd(dim, m, oracle_lib):
    rng = np.random.default_rng(20 + dim)
    n, L, ns = 50000, 1.0, 3
    X = rng.uniform(0, L, (n, dim)).astype(np.float32)
    X[:50] = 0.0
    X[50:100] = L
    sp = rng.integers(0, ns, n).astype(np.uint8)
    counts, totals = oracle.species_hist(dim, L, X, sp, ns, m)
    assert counts.shape == (ns, m ** dim)
    assert np.array_equal(totals, np.bincount(sp, minlength=ns))
    assert counts.sum() == n
    edges = np.linspace(0, L, m + 1)
    s = X.astype(np.float64) * m / L
    near = (np.abs(s - np.rint(s)) < 1e-4).any(1) & (X > 0).all(1) & (X < L).all(1)
    keep = ~near
    ref_counts, _ = oracle.species_hist(dim, L, X[keep], sp[keep], ns, m)
    for k in range(ns):
        sel = keep & (sp == k)
        h, _ = np.histogramdd(X[sel].astype(np.float64), bins=[edges] * dim)
        # histogramdd indexes [x][y][z]; the oracle stores x fastest
        assert np.array_equal(ref_counts[k], h.T.reshape(-1).astype(np.uint32))


def test_species_hist_hand_placed(oracle_lib):
    m, L = 10, 2.0
    X = np.array([[0.7, 0.3], [0.71, 0.39], [1.99, 0.0], [2.0, 2.0]], np.float32)
    sp = np.array([0, 0, 1, 1], np.uint8)
    counts, totals = oracle.species_hist(2, L, X, sp, 2, m)
    # (0.7, 0.3) -> bins (3, 1) -> index 1 * 10 + 3
    assert counts[0, 13] == 2 and counts[0].sum() == 2
    assert counts[1, 9] == 1            # (1.99, 0) -> (9, 0)
    assert counts[1, 99] == 1           # upper corner -> last bin
    assert list(totals) == [2, 2]


def test_field_mean(oracle_lib):
    c = np.arange(12, dtype=np.float32)
    assert np.allclose(oracle.field_mean(c, 3), [4, 5, 6, 7])
