"""Pins of the oracle's pair and update variants (Sect. 2.2 and Sect. 4):

* pair forces are minus the gradient of the pair energy: central finite
  differences of U = sum_pairs u(r) (harmonic (k/2)(d - r)^2; exponential
  k exp(-r/d) cut at pot_range * d) match F to FD accuracy;
* the exponential force of a lone pair has the closed form (k/d) e^{-r/d};
* tamed Euler (eq. sde_ETamed): the pair drift step F dt / (1 + |F| dt) is
  shorter than one however steep the force, and tends to the
  Euler-Maruyama step F dt as dt -> 0;
* hard-sphere overlap correction: a lone overlapping pair ends 2d - r apart
  with shares D_i / (D_i + D_j) of the push (equal halves for equal D, all
  of it for the mobile partner of an immobile obstacle, nothing for two
  obstacles); sum_i X_i / D_i is unchanged by the correction;
* a hard-sphere step is the force-free update followed by the correction.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _wl(species, n, potential=0, tamed=False, pot_range=3.0, k=50.0, dt=1e-4, L=1.0, grid_n=8,
        periodic=True):
    return W.Workload("v", 2, periodic, L, grid_n, dt, k, 0.0, 0.0, 1, tuple(species),
                      (W.Instance(n, 3),), potential=potential, tamed=tamed, pot_range=pot_range,
                      c0="zero")


def _energy(p, X, sp, potential):
    U = 0.0
    n = len(X)
    for i in range(n):
        for j in range(i + 1, n):
            d = 0.5 * (p.diam[sp[i]] + p.diam[sp[j]])
            dx = X[j] - X[i]
            dx -= np.rint(dx)
            r = math.sqrt((dx ** 2).sum())
            if potential == 0 and r < d:
                U += 0.5 * p.k * (d - r) ** 2
            if potential == 1 and r < p.pot_range * d:
                U += p.k * math.exp(-r / d)
    return U


@pytest.mark.parametrize("potential", [0, 1])
def test_force_is_minus_energy_gradient(potential, oracle_lib):
    sp = (W.Species(0.05, 0.0, 0.0, 0.0, 0.0), W.Species(0.08, 0.0, 0.0, 0.0, 0.0))
    w = _wl(sp, 12, potential=potential)
    p = oracle.params(w)
    rng = np.random.default_rng(40 + potential)
    X = 0.45 + 0.1 * rng.uniform(size=(12, 2))
    s = rng.integers(0, 2, 12).astype(np.uint8)
    F = oracle.forces(p, X, s)
    h = 1e-6
    for i in range(12):
        for a in range(2):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, a] += h
            Xm[i, a] -= h
            g = (_energy(p, Xp, s, potential) - _energy(p, Xm, s, potential)) / (2 * h)
            assert abs(F[i, a] + g) < 1e-5 * max(1.0, abs(g)), (i, a, F[i, a], -g)
    assert np.abs(F.sum(0)).max() < 1e-9 * np.abs(F).max()


def test_exponential_pair_closed_form_and_range(oracle_lib):
    d, k = 0.02, 3.0
    w = _wl((W.Species(d, 0.0, 0.0, 0.0, 0.0),), 2, potential=1, k=k, pot_range=2.5)
    p = oracle.params(w)
    for r in (0.0005, 0.01, 0.03, 0.0499):
        X = np.array([[0.5, 0.5], [0.5 + r * 0.6, 0.5 + r * 0.8]])
        F = oracle.forces(p, X, np.zeros(2, np.uint8))
        mag = (k / d) * math.exp(-r / d)
        np.testing.assert_allclose(F[0], -mag * np.array([0.6, 0.8]), rtol=1e-12)
        np.testing.assert_allclose(F[1], mag * np.array([0.6, 0.8]), rtol=1e-12)
    X = np.array([[0.5, 0.5], [0.5 + 0.0501, 0.5]])  # beyond 2.5 d
    assert np.all(oracle.forces(p, X, np.zeros(2, np.uint8)) == 0)


def test_tamed_step_bounded_and_consistent(oracle_lib):
    d = 0.02
    sp = (W.Species(d, 0.0, 0.0, 0.0, 0.0),)
    X0 = np.array([[5.0, 5.0], [5.0 + 0.001, 5.0]])
    for k in (1e3, 1e6, 1e9):
        for dt in (1e-3, 1e-6):
            w = _wl(sp, 2, potential=0, tamed=True, k=k, dt=dt, L=10.0)  # no wrap
            p = oracle.params(w)
            F = oracle.forces(p, X0, np.zeros(2, np.uint8))
            X1, _, _ = oracle.run(p, X0, np.zeros(2, np.uint8), np.zeros(w.n_nodes), 0, 1)
            step = X1 - X0
            assert np.all(np.linalg.norm(step, axis=1) < 1.0)
            nf = np.linalg.norm(F, axis=1, keepdims=True)
            np.testing.assert_allclose(step, F * dt / (1 + nf * dt), rtol=1e-10, atol=1e-15)
    # small dt: tamed and Euler-Maruyama steps agree to first order
    w0 = _wl(sp, 2, potential=0, tamed=False, k=10.0, dt=1e-7, L=10.0)
    w1 = _wl(sp, 2, potential=0, tamed=True, k=10.0, dt=1e-7, L=10.0)
    a, _, _ = oracle.run(oracle.params(w0), X0, np.zeros(2, np.uint8), np.zeros(64), 0, 1)
    b, _, _ = oracle.run(oracle.params(w1), X0, np.zeros(2, np.uint8), np.zeros(64), 0, 1)
    assert np.abs((a - X0)[:, 0] / (b - X0)[:, 0] - 1).max() < 1e-6


@pytest.mark.parametrize("Di,Dj", [(1.0, 1.0), (1.0, 3.0), (0.0, 2.0), (0.0, 0.0)])
def test_hard_sphere_pair(Di, Dj, oracle_lib):
    sp = (W.Species(0.02, Di, 0.0, 0.0, 0.0), W.Species(0.04, Dj, 0.0, 0.0, 0.0))
    w = _wl(sp, 2, potential=2)
    p = oracle.params(w)
    r, u = 0.01, np.array([0.6, 0.8])
    X = np.array([[0.5, 0.5], [0.5, 0.5] + r * u])
    Y = oracle.hs_correct(p, X, np.array([0, 1], np.uint8))
    d = 0.03
    dp = d - r
    if Di + Dj == 0:
        np.testing.assert_array_equal(Y, X)
        return
    np.testing.assert_allclose(Y[0], X[0] - 2 * dp * Di / (Di + Dj) * u, atol=1e-15)
    np.testing.assert_allclose(Y[1], X[1] + 2 * dp * Dj / (Di + Dj) * u, atol=1e-15)
    assert abs(np.linalg.norm(Y[1] - Y[0]) - (2 * d - r)) < 1e-14


def test_hard_sphere_weighted_centre_invariant(oracle_lib):
    sp = (W.Species(0.03, 1.0, 0.0, 0.0, 0.0), W.Species(0.05, 0.25, 0.0, 0.0, 0.0))
    w = _wl(sp, 300, potential=2)
    p = oracle.params(w)
    rng = np.random.default_rng(8)
    X = 0.3 + 0.4 * rng.uniform(size=(300, 2))   # dense, away from the seam
    s = rng.integers(0, 2, 300).astype(np.uint8)
    Y = oracle.hs_correct(p, X, s)
    Dv = np.array([1.0, 0.25])[s][:, None]
    np.testing.assert_allclose((Y / Dv).sum(0), (X / Dv).sum(0), rtol=1e-12)
    assert np.abs(Y - X).max() > 1e-3


def test_hard_sphere_step_is_free_update_then_correction(oracle_lib):
    sp = (W.Species(0.03, 0.5, 0.0, 0.0, 0.0),)
    n = 400
    w = _wl(sp, n, potential=2, k=123.0, dt=1e-4)
    p = oracle.params(w)
    X0 = np.random.default_rng(9).uniform(0, 1, (n, 2))
    X1, _, _ = oracle.run(p, X0, np.zeros(n, np.uint8), np.zeros(w.n_nodes), 0, 1)
    xi = oracle.normals(p, 0, np.arange(n, dtype=np.uint32))[:, :2]
    Xf = np.mod(X0 + math.sqrt(2 * 0.5 * 1e-4) * xi, 1.0)
    np.testing.assert_allclose(X1, oracle.hs_correct(p, Xf, np.zeros(n, np.uint8)), atol=1e-14)
