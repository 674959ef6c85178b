"""Pins of the oracle's boundary closure (no-flux walls and the periodic
seam; boundary conditions of Sect. 2, reflection listing of Sect. 3.2).

* a deterministic agent (D = 0) driven across a wall by chemotaxis on a
  linear field lands at the mirror point of where the update put it
  (x < 0 -> -x, x > L -> 2L - x); the expected value is worked out here by
  hand from the interpolated centred-difference gradient, on every axis of
  2D and 3D boxes;
* reflected free diffusion: with one specular reflection per step the walk
  X_{n+1} = |X_n + xi| has, for symmetric xi, the same law as |x0 + S_n|
  (the folded normal), so its mean and mean-squared displacement near a
  wall have closed forms; a uniform start stays uniform;
* the periodic edge rule: a position that rounds to L after the wrap is
  taken to 0, so every periodic coordinate lies in [0, L).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _walls(dim, species, n, grid_n, dt, periodic=False, seed=77):
    return W.Workload("b", dim, periodic, 1.0, grid_n, dt, 0.0, 0.0, 0.0, 1, tuple(species),
                      (W.Instance(n, seed),), c0="zero")


def _linear_field(w, axis, sign):
    """c = x_axis (sign +1) or 1 - x_axis (sign -1) on the node grid, x fastest."""
    xs = W.node_coords(w)
    grids = np.meshgrid(*([xs] * w.dim), indexing="ij")   # grids[a][i0, i1, ...] = xs[i_a]
    # C order [z][y][x]: axis a of the position is array axis dim - 1 - a
    coord = grids[w.dim - 1 - axis]
    c = coord if sign > 0 else 1.0 - coord
    return np.ascontiguousarray(c).reshape(-1)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("side", ["low", "high"])
def test_drift_across_wall_lands_at_mirror_point(dim, side, oracle_lib):
    G, dt, chi = 17, 0.1, 2.0
    h = 1.0 / (G - 1)
    for axis in range(dim):
        w = _walls(dim, [W.Species(0.01, 0.0, chi, 0.0, 0.0)], 1, G, dt)
        p = oracle.params(w)
        X = np.full((1, dim), 0.5)
        if side == "high":
            # c = x_axis: interior node gradients 1, wall nodes 0 (mirror
            # ghost); in the last cell the interpolated gradient is 1 - t
            x0, t = 1.0 - 0.75 * h, 0.25
            c = _linear_field(w, axis, +1)
            g = 1.0 - t
        else:
            # c = 1 - x_axis: interior gradients -1, wall node 0; in the
            # first cell the interpolated gradient is -t
            x0, t = 0.25 * h, 0.25
            c = _linear_field(w, axis, -1)
            g = -t
        X[0, axis] = x0
        X1, _, _ = oracle.run(p, X, np.zeros(1, np.uint8), c, 0, 1)
        moved = x0 + dt * chi * g
        assert (moved > 1.0) if side == "high" else (moved < 0.0)
        mirror = 2.0 - moved if side == "high" else -moved
        expect = np.full(dim, 0.5)
        expect[axis] = mirror
        np.testing.assert_allclose(X1[0], expect, rtol=0, atol=1e-14)


def _folded_mean(a, s):
    """E|a + s Z| for Z ~ N(0, 1)."""
    return s * math.sqrt(2 / math.pi) * math.exp(-a * a / (2 * s * s)) + \
        a * (1 - 2 * 0.5 * math.erfc(a / (s * math.sqrt(2))))


@pytest.mark.parametrize("dim", [2, 3])
def test_reflected_diffusion_near_a_wall_is_folded_normal(dim, oracle_lib):
    """Agents start at distance a from the lower wall of axis 0; after n
    steps X_0 has the law of |a + S_n|, S_n ~ N(0, 2 D n dt), far from the
    other wall.  Mean and mean-squared displacement within 5 standard
    errors.  A clamp at the wall (x < 0 -> 0) gives the law of the running
    maximum instead, about 0.5 step lengths lower at n = 10."""
    n, D, dt, steps, a = 20000, 0.5, 1e-4, 10, 0.005
    w = _walls(dim, [W.Species(0.01, D, 0.0, 0.0, 0.0)], n, 9, dt)
    p = oracle.params(w)
    rng = np.random.default_rng(11)
    X = rng.uniform(0.3, 0.7, (n, dim))
    X[:, 0] = a
    X1, _, _ = oracle.run(p, X, np.zeros(n, np.uint8), np.zeros(w.n_nodes), 0, steps)
    s = math.sqrt(2 * D * dt * steps)
    m1 = _folded_mean(a, s)
    m2 = a * a + s * s                      # E (a + S)^2 = E X^2
    msd = m2 - 2 * a * m1 + a * a           # E (X - a)^2
    x = X1[:, 0]
    se1 = math.sqrt(m2 - m1 * m1) / math.sqrt(n)
    assert abs(x.mean() - m1) < 5 * se1
    d2 = (x - a) ** 2
    assert abs(d2.mean() - msd) < 5 * d2.std() / math.sqrt(n)
    assert x.min() >= 0.0


@pytest.mark.parametrize("dim", [2, 3])
def test_reflected_diffusion_keeps_uniform_density(dim, oracle_lib):
    """The uniform law is invariant under the reflected walk: per-axis
    histograms of 20 bins stay within 5 sigma of n/20 after many wall hits."""
    n, D, dt, steps, nb = 20000, 1.0, 1e-3, 30, 20
    w = _walls(dim, [W.Species(0.001, D, 0.0, 0.0, 0.0)], n, 9, dt)
    p = oracle.params(w)
    X = np.random.default_rng(12).uniform(0.0, 1.0, (n, dim))
    X1, _, _ = oracle.run(p, X, np.zeros(n, np.uint8), np.zeros(w.n_nodes), 0, steps)
    assert X1.min() >= 0.0 and X1.max() <= 1.0
    e = n / nb
    sd = math.sqrt(n * (1 / nb) * (1 - 1 / nb))
    for ax in range(dim):
        h, _ = np.histogram(X1[:, ax], bins=nb, range=(0.0, 1.0))
        assert np.abs(h - e).max() < 5 * sd, (ax, h)


@pytest.mark.parametrize("dim", [2, 3])
def test_periodic_wrap_of_a_position_that_rounds_to_L(dim, oracle_lib):
    """An agent at x = 0 moved by -delta with delta below half an ulp of L:
    x - L floor(x / L) = L - delta rounds to L in FP64, and the edge rule
    takes it to 0, not L.  A position just inside L stays where it is."""
    G = 16
    h = 1.0 / G
    w = _walls(dim, [W.Species(0.01, 0.0, 1.0, 0.0, 0.0)], 1, G, 1.0, periodic=True)
    xs = W.node_coords(w)
    grids = np.meshgrid(*([xs] * dim), indexing="ij")
    for axis in range(dim):
        # c = -sin(2 pi x_axis): the centred-difference gradient at node 0 is
        # -sin(2 pi h) / h, so the drift at x = 0 is chi times that
        c = np.ascontiguousarray(-np.sin(2 * np.pi * grids[dim - 1 - axis])).reshape(-1)
        g0 = -math.sin(2 * math.pi * h) / h
        for delta, expect in ((2.0 ** -56, 0.0), (1e-10, 1.0 - 1e-10)):
            chi = delta / -g0
            ww = _walls(dim, [W.Species(0.01, 0.0, chi, 0.0, 0.0)], 1, G, 1.0, periodic=True)
            p = oracle.params(ww)
            X = np.full((1, dim), 0.5)
            X[0, axis] = 0.0
            X1, _, _ = oracle.run(p, X, np.zeros(1, np.uint8), c, 0, 1)
            assert 0.0 <= X1[0, axis] < 1.0
            assert X1[0, axis] == pytest.approx(expect, abs=1e-15), (axis, delta, X1)
            if expect == 0.0:
                assert X1[0, axis] == 0.0
