"""Pins of the oracle's grid operators (Sect. 2.3 and 3.5 of the paper).

* interpolation: exact on affine fields, reproduces node values at nodes;
* deposit: conserves total source (sum of sigma_l h^d v_l = sum_i k_s);
* duality: <deposit(q), f> = <q, interp(f)> (the two are transposes);
* central-difference gradient: exact on quadratics in the interior;
* PDE: exact discrete decay of a Fourier mode, mass conservation under
  zero flux without sources, convergence to the continuum heat kernel
  with decay (the Green's function G_gamma of Sect. 2.3).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _w(dim, periodic, n=17, **kw):
    base = dict(dt=1e-5, k=0.0, D_c=1.0, gamma=0.0, steps=1)
    base.update(kw)
    return W.Workload("g", dim, periodic, 1.0, n, base["dt"], base["k"], base["D_c"],
                      base["gamma"], base["steps"],
                      (W.Species(0.01, 1.0, 1.0, 1.0, 0.5), W.Species(0.01, 1.0, 0.0, 0.0, 2.0)),
                      (W.Instance(1, 5),))


def _nodes(w):
    xs = W.node_coords(w)
    g = np.meshgrid(*([xs] * w.dim), indexing="ij")
    return [np.ascontiguousarray(a.T).reshape(-1) for a in g]  # x fastest


@pytest.mark.parametrize("dim", [2, 3])
def test_interp_exact_on_affine_walls(dim, oracle_lib):
    w = _w(dim, False, n=9)
    p = oracle.params(w)
    coef = np.array([0.3, -1.7, 2.2][:dim])
    nodes = _nodes(w)
    f = 0.5 + sum(c * x for c, x in zip(coef, nodes))
    X = np.random.default_rng(0).uniform(0, 1, (500, dim))
    X[:5] = 1.0  # upper wall corner cell
    X[5:10] = 0.0
    got = oracle.interp(p, f, X)
    np.testing.assert_allclose(got, 0.5 + X @ coef, rtol=0, atol=1e-13)
    # multilinear also reproduces x*y products exactly on [0,L]^d
    f2 = nodes[0] * nodes[1]
    np.testing.assert_allclose(oracle.interp(p, f2, X), X[:, 0] * X[:, 1], atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_interp_node_values_periodic(dim, oracle_lib):
    w = _w(dim, True, n=8)
    p = oracle.params(w)
    f = np.random.default_rng(1).standard_normal(8 ** dim)
    nodes = np.stack(_nodes(w), 1)
    np.testing.assert_allclose(oracle.interp(p, f, nodes), f, atol=1e-14)
    # inside the seam cell the interpolant blends the last node with node 0
    x = np.zeros((1, dim)) + 0.0
    x[0, 0] = 7.5 / 8
    l_last = 7
    np.testing.assert_allclose(oracle.interp(p, f, x)[0], 0.5 * (f[l_last] + f[0]), atol=1e-14)


@pytest.mark.parametrize("dim,periodic", [(2, True), (2, False), (3, True), (3, False)])
def test_deposit_mass_and_duality(dim, periodic, oracle_lib):
    w = _w(dim, periodic, n=11)
    p = oracle.params(w)
    rng = np.random.default_rng(2)
    n = 3000
    X = rng.uniform(0, 1, (n, dim))
    X[:20] = 0.0 if not periodic else 0.999999
    if not periodic:
        X[20:40] = 1.0
    sp = rng.integers(0, 2, n).astype(np.uint8)
    Ss, Su = oracle.deposit(p, X, sp)
    src = np.array([1.0, 0.0])[sp].sum()
    upt = np.array([0.5, 2.0])[sp].sum()
    assert abs(Ss.sum() - src) <= 1e-12 * src
    assert abs(Su.sum() - upt) <= 1e-12 * upt
    # transpose identity with an arbitrary field f
    f = rng.standard_normal(len(Ss))
    lhs = (Ss * f).sum()
    rhs = (np.array([1.0, 0.0])[sp] * oracle.interp(p, f, X)).sum()
    assert abs(lhs - rhs) <= 1e-12 * np.abs(f).sum()


@pytest.mark.parametrize("dim,periodic", [(2, True), (2, False), (3, False)])
def test_gradient_central_difference(dim, periodic, oracle_lib):
    w = _w(dim, periodic, n=12)
    p = oracle.params(w)
    nodes = _nodes(w)
    h = 1.0 / 12 if periodic else 1.0 / 11
    if periodic:
        k = 2 * np.pi
        c = np.sin(k * nodes[0]) + np.cos(k * nodes[1])
        g = oracle.gradient(p, c)
        # centred difference of a Fourier mode: exact factor sin(kh)/h
        np.testing.assert_allclose(g[0], np.sin(k * h) / h * np.cos(k * nodes[0]), atol=1e-12)
        np.testing.assert_allclose(g[1], -np.sin(k * h) / h * np.sin(k * nodes[1]), atol=1e-12)
    else:
        c = nodes[0] ** 2 + 3 * nodes[1]
        g = oracle.gradient(p, c)
        ix = np.rint(nodes[0] / h).astype(int)
        iy = np.rint(nodes[1] / h).astype(int)
        inner = (ix > 0) & (ix < 11)
        np.testing.assert_allclose(g[0][inner], 2 * nodes[0][inner], atol=1e-12)
        assert np.all(g[0][~inner] == 0.0)  # mirror ghost: zero normal gradient on walls
        inner_y = (iy > 0) & (iy < 11)
        np.testing.assert_allclose(g[1][inner_y], 3.0, atol=1e-12)
        assert np.all(g[1][~inner_y] == 0.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_pde_fourier_mode_exact_decay(dim, oracle_lib):
    n = 32
    w = _w(dim, True, n=n, dt=2e-5, gamma=0.3, D_c=1.0)
    p = oracle.params(w)
    p.n_sub = 2
    nodes = _nodes(w)
    mode = np.ones_like(nodes[0])
    for x in nodes:
        mode = mode * np.sin(2 * np.pi * x)
    A, B = 0.7, 1.3
    c = A * mode + B
    z = np.zeros(n ** dim)
    c1 = oracle.pde(p, c, z, z)
    h = 1.0 / n
    dts = p.dt / p.n_sub
    lam = -dim * 4 / h**2 * math.sin(math.pi * h) ** 2
    amp = A * (1 + dts * (p.D_c * lam - p.gamma)) ** p.n_sub
    mean = B * (1 - dts * p.gamma) ** p.n_sub
    np.testing.assert_allclose(c1, amp * mode + mean, rtol=0, atol=1e-12)


@pytest.mark.parametrize("dim,periodic", [(2, True), (2, False), (3, True), (3, False)])
def test_pde_mass_conserved_without_sources(dim, periodic, oracle_lib):
    w = _w(dim, periodic, n=13, dt=1e-4, gamma=0.0)
    p = oracle.params(w)
    p.n_sub = 3
    rng = np.random.default_rng(3)
    c = rng.uniform(0.5, 2.0, 13 ** dim)
    z = np.zeros_like(c)
    vol = np.ones_like(c)
    if not periodic:
        idx = np.indices((13,) * dim).reshape(dim, -1)
        for a in range(dim):
            vol *= np.where((idx[a] == 0) | (idx[a] == 12), 0.5, 1.0)
    m0 = (vol * c).sum()
    for _ in range(5):
        c = oracle.pde(p, c, z, z)
    assert abs((vol * c).sum() - m0) <= 1e-12 * m0


def test_pde_sources_and_uptake(oracle_lib):
    # one node with deposited source S and uptake U: the update is explicit
    w = _w(2, True, n=8, dt=1e-3, gamma=0.25, D_c=0.0)
    p = oracle.params(w)
    p.n_sub = 1
    c = np.full(64, 2.0)
    Ss = np.zeros(64); Su = np.zeros(64)
    Ss[9] = 0.5; Su[9] = 0.25
    c1 = oracle.pde(p, c, Ss, Su)
    h2 = (1.0 / 8) ** 2
    expect = 2.0 + p.dt * (0.5 / h2 - 0.25 / h2 * 2.0 - 0.25 * 2.0)
    assert abs(c1[9] - expect) < 1e-13
    assert np.allclose(np.delete(c1, 9), 2.0 * (1 - p.dt * 0.25), atol=1e-14)


def test_pde_converges_to_heat_kernel(oracle_lib):
    """A narrow Gaussian evolves like G_gamma: variance s0^2 + 2 D_c t per
    axis and total mass times exp(-gamma t); error shrinks ~ h^2."""
    errs = []
    D_c, gam, s0, T = 1.0, 0.5, 0.05, 2e-3
    for n in (32, 64):
        dt = 0.2 * (1.0 / n) ** 2 / D_c
        steps = int(round(T / dt))
        w = _w(2, True, n=n, dt=T / steps, gamma=gam, D_c=D_c)
        p = oracle.params(w)
        p.n_sub = 1
        x, y = _nodes(w)
        r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2
        c = np.exp(-r2 / (2 * s0**2)) / (2 * np.pi * s0**2)
        z = np.zeros_like(c)
        for _ in range(steps):
            c = oracle.pde(p, c, z, z)
        s2 = s0**2 + 2 * D_c * T
        exact = math.exp(-gam * T) * np.exp(-r2 / (2 * s2)) / (2 * np.pi * s2)
        errs.append(np.abs(c - exact).max() / exact.max())
    assert errs[0] < 0.05
    assert errs[1] < errs[0] / 3.0  # second order in space (dt ~ h^2)
