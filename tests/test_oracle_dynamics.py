"""Pins of whole oracle steps against closed forms and invariants.

* free diffusion: MSD(t) = 2 d D t (the pure-diffusion case of the MSD
  experiment, Fig. 3 (1));
* constant chemotactic drift with c = x: mean displacement chi t e_x and
  MSD = 2 d D t + chi^2 t^2 (Fig. 3 (2));
* pure repulsion (D = 0, chi = 0): the overlap energy sum (k/2)(d - r)^2
  never increases ("no overlap growth");
* reflecting walls keep every agent in [0, L]^d;
* splitting order of one step (drift from c^n at X^n, deposit at X^{n+1},
  PDE with those sources), checked on one agent by hand.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _wl(dim, periodic, species, n, grid_n=16, dt=1e-4, k=0.0, D_c=0.0, gamma=0.0, c0="zero",
        seed=77):
    return W.Workload("d", dim, periodic, 1.0, grid_n, dt, k, D_c, gamma, 1, tuple(species),
                      (W.Instance(n, seed),), c0=c0)


def _minimg(d):
    return d - np.rint(d)


@pytest.mark.parametrize("dim", [2, 3])
def test_free_diffusion_msd(dim, oracle_lib):
    D, dt, steps, n = 0.7, 1e-4, 40, 20000
    w = _wl(dim, True, [W.Species(0.01, D, 0.0, 0.0, 0.0)], n, dt=dt)
    p = oracle.params(w)
    rng = np.random.default_rng(5)
    X = rng.uniform(0, 1, (n, dim))
    sp = np.zeros(n, np.uint8)
    c = np.zeros(w.n_nodes)
    disp = np.zeros_like(X)
    st = 0
    for s in range(steps):
        Xn, c, st = oracle.step(p, X, sp, c, st)
        disp += _minimg(Xn - X)
        X = Xn
    t = steps * dt
    msd = (disp ** 2).sum(1)
    expect = 2 * dim * D * t
    sigma = expect * math.sqrt(2.0 / dim) / math.sqrt(n)
    assert abs(msd.mean() - expect) < 5 * sigma


def test_constant_drift_walls(oracle_lib):
    D, chi, dt, steps, n, G = 0.01, 1.0, 1e-3, 10, 20000, 33
    w = _wl(2, False, [W.Species(0.01, D, chi, 0.0, 0.0)], n, grid_n=G, dt=dt)
    p = oracle.params(w)
    xs = W.node_coords(w)
    c = np.tile(xs, G)  # c(x, y) = x, x fastest
    rng = np.random.default_rng(6)
    X = rng.uniform(0.35, 0.65, (n, 2))
    X0 = X.copy()
    sp = np.zeros(n, np.uint8)
    X1, c1, _ = oracle.run(p, X, sp, c, 0, steps)
    assert np.array_equal(c1, c)  # D_c = gamma = 0 and no sources
    t = steps * dt
    d = X1 - X0
    assert abs(d[:, 0].mean() - chi * t) < 5 * math.sqrt(2 * D * t / n)
    assert abs(d[:, 1].mean()) < 5 * math.sqrt(2 * D * t / n)
    msd = (d ** 2).sum(1).mean()
    expect = 4 * D * t + chi**2 * t**2
    assert abs(msd - expect) < 5 * expect * math.sqrt(1.0 / n) * 2


def _energy(X, k, d):
    from scipy.spatial import cKDTree
    pairs = cKDTree(X, boxsize=1.0).query_pairs(d, output_type="ndarray")
    dx = _minimg(X[pairs[:, 1]] - X[pairs[:, 0]])
    r = np.sqrt((dx ** 2).sum(1))
    return 0.5 * k * ((d - r) ** 2).sum()


@pytest.mark.parametrize("dim", [2, 3])
def test_pure_repulsion_energy_never_increases(dim, oracle_lib):
    n, d, k, dt = 3000, 0.02 if dim == 2 else 0.05, 100.0, 1e-4
    w = _wl(dim, True, [W.Species(d, 0.0, 0.0, 0.0, 0.0)], n, dt=dt, k=k)
    p = oracle.params(w)
    X = np.random.default_rng(8).uniform(0, 1, (n, dim)) * 0.5
    sp = np.zeros(n, np.uint8)
    c = np.zeros(w.n_nodes)
    E = [_energy(X, k, d)]
    st = 0
    for _ in range(15):
        X, c, st = oracle.step(p, X, sp, c, st)
        E.append(_energy(X, k, d))
    assert E[0] > 0
    assert all(b <= a * (1 + 1e-12) for a, b in zip(E, E[1:]))
    assert E[-1] < 0.9 * E[0]


def test_walls_keep_agents_inside(oracle_lib):
    n = 5000
    w = _wl(2, False, [W.Species(0.01, 5.0, 0.0, 1.0, 0.0)], n, dt=1e-3, k=100.0, D_c=1.0)
    p = oracle.params(w)
    X = np.random.default_rng(9).uniform(0, 1, (n, 2))
    X[:100] = 0.0
    X[100:200] = 1.0
    sp = np.zeros(n, np.uint8)
    c = np.ones(w.n_nodes)
    st = 0
    for _ in range(10):
        X, c, st = oracle.step(p, X, sp, c, st)
        assert X.min() >= 0.0 and X.max() <= 1.0


def test_step_order_single_agent(oracle_lib):
    """D = 0 so the step is deterministic: X1 = X0 + dt chi grad_h c^0 (X0),
    then c^1 = c^0 + dt (D_c Lap c^0 + sigma(X1) - gamma c^0)."""
    G, dt, chi, gam, Dc = 9, 1e-3, 2.0, 0.5, 0.3
    w = _wl(2, False, [W.Species(0.01, 0.0, chi, 3.0, 0.0)], 1, grid_n=G, dt=dt, D_c=Dc,
            gamma=gam)
    p = oracle.params(w)
    p.n_sub = 1
    h = 1.0 / (G - 1)
    xs = W.node_coords(w)
    X_, Y_ = np.meshgrid(xs, xs, indexing="xy")  # [y][x]
    c0 = (X_ ** 2 + 0.5 * Y_).reshape(-1)       # x fastest
    x0 = np.array([[0.40, 0.30]])
    X1, c1, st = oracle.step(p, x0, np.zeros(1, np.uint8), c0, 41)
    assert st == 42
    # hand-computed drift: central differences of x^2 are exact (2x) and of
    # 0.5 y exact (0.5) at interior nodes; bilinear of 2x is 2x
    drift = chi * np.array([2 * 0.40, 0.5])
    np.testing.assert_allclose(X1[0], x0[0] + dt * drift, atol=1e-14)
    # deposit at X1, not at x0
    ix, iy = int(X1[0, 0] // h), int(X1[0, 1] // h)
    tx, ty = X1[0, 0] / h - ix, X1[0, 1] / h - iy
    S = np.zeros((G, G))
    S[iy, ix] += (1 - tx) * (1 - ty); S[iy, ix + 1] += tx * (1 - ty)
    S[iy + 1, ix] += (1 - tx) * ty; S[iy + 1, ix + 1] += tx * ty
    S *= 3.0
    c = c0.reshape(G, G)
    cp = np.pad(c, 1, mode="reflect")  # mirror ghost nodes
    lap = (cp[1:-1, 2:] + cp[1:-1, :-2] + cp[2:, 1:-1] + cp[:-2, 1:-1] - 4 * c) / h**2
    vol = np.ones((G, G))
    vol[0, :] *= 0.5; vol[-1, :] *= 0.5; vol[:, 0] *= 0.5; vol[:, -1] *= 0.5
    expect = c + dt * (Dc * lap + S / (h * h * vol) - gam * c)
    np.testing.assert_allclose(c1.reshape(G, G), expect, rtol=1e-12, atol=1e-12)
