"""Pins of the oracle's Gaussian kernel density deposit (Sect. 2.3 and the
density loop of Sect. 3.5): K_eps(x) = (2 pi eps^2)^(-d/2) exp(-|x|^2/(2 eps^2)),
bandwidth eps = the species' diameter, truncated at kde_radius * eps.

* the lattice sum h^d sum_l K(p_l - X) of a Gaussian wider than the node
  spacing equals its integral up to exp(-2 pi^2 eps^2 / h^2) (Poisson
  summation), so the mass is 1 for a wide truncation and the closed-form
  Gaussian mass inside radius kappa * eps otherwise (2D: 1 - exp(-kappa^2/2);
  3D: erf(kappa/sqrt 2) - sqrt(2/pi) kappa exp(-kappa^2/2));
* the second moment is d eps^2 (pins the 2 eps^2 of the exponent);
* the torus wraps (an agent on the seam keeps its mass and symmetry);
* with walls there is no image: an agent on a wall keeps half its mass on
  the trapezoid-weighted grid;
* the peak at an agent on a node is (2 pi eps^2)^(-d/2) source;
* a whole step with D = chi = 0 uses the kernel density at X^{n+1}.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _wl(dim, periodic, eps, grid_n, species=None, kappa=6.0, dt=1e-3, D_c=0.0, gamma=0.0):
    sp = species or (W.Species(eps, 0.0, 0.0, 1.0, 0.5),)
    return W.Workload("k", dim, periodic, 1.0, grid_n, dt, 0.0, D_c, gamma, 1, tuple(sp),
                      (W.Instance(1, 5),), deposit_kernel=1, kde_radius=kappa, c0="zero")


def _nodes(w):
    xs = W.node_coords(w)
    g = np.meshgrid(*([xs] * w.dim), indexing="ij")
    return np.stack([a.T.reshape(-1) for a in g], 1)  # x fastest


def _mass_inside(dim, kappa):
    if dim == 2:
        return 1 - math.exp(-kappa ** 2 / 2)
    return math.erf(kappa / math.sqrt(2)) - math.sqrt(2 / math.pi) * kappa * math.exp(-kappa ** 2 / 2)


@pytest.mark.parametrize("dim,G", [(2, 64), (3, 32)])
def test_mass_and_second_moment_on_the_torus(dim, G, oracle_lib):
    h = 1.0 / G
    eps = 2.5 * h
    w = _wl(dim, True, eps, G)
    p = oracle.params(w)
    rng = np.random.default_rng(dim)
    for X in (rng.uniform(0, 1, (1, dim)), np.full((1, dim), 0.001)):  # interior, seam
        sig, ups = oracle.deposit_kde(p, X, np.zeros(1, np.uint8))
        assert abs(sig.sum() * h ** dim - 1.0) < 1e-6
        np.testing.assert_allclose(ups, 0.5 * sig, rtol=1e-15)
        d = _nodes(w) - X
        d -= np.rint(d)
        m2 = (sig * (d ** 2).sum(1)).sum() * h ** dim
        assert abs(m2 - dim * eps ** 2) < 1e-6 * eps ** 2 * 10
        # first moment zero about the agent (symmetry, across the seam too)
        assert np.abs((sig[:, None] * d).sum(0) * h ** dim).max() < 1e-9


@pytest.mark.parametrize("dim,kappa", [(2, 1.0), (2, 2.0), (3, 1.5)])
def test_truncated_mass(dim, kappa, oracle_lib):
    G = 128 if dim == 2 else 64
    h = 1.0 / G
    eps = 10 * h
    w = _wl(dim, True, eps, G, kappa=kappa)
    p = oracle.params(w)
    sig, _ = oracle.deposit_kde(p, np.full((1, dim), 0.5 + 0.37 * h), np.zeros(1, np.uint8))
    mass = sig.sum() * h ** dim
    assert abs(mass - _mass_inside(dim, kappa)) < 0.02 * _mass_inside(dim, kappa)
    assert mass < _mass_inside(dim, kappa + 0.2)


def test_peak_value_and_per_species_bandwidth(oracle_lib):
    G = 100
    h = 1.0 / G
    sp = (W.Species(0.03, 0.0, 0.0, 2.0, 0.0), W.Species(0.06, 0.0, 0.0, 0.0, 1.0))
    w = _wl(2, True, None, G, species=sp)
    p = oracle.params(w)
    X = np.array([[0.5, 0.5], [0.2, 0.7]])
    sig, ups = oracle.deposit_kde(p, X, np.array([0, 1], np.uint8))
    l0 = 50 * G + 50
    assert abs(sig[l0] - 2.0 / (2 * math.pi * 0.03 ** 2)) < 1e-9 * sig[l0]
    d = _nodes(w)
    for vals, x, eps in ((sig / 2.0, X[0], 0.03), (ups, X[1], 0.06)):
        dd = d - x
        dd -= np.rint(dd)
        assert abs(vals.sum() * h * h - 1) < 1e-6
        assert abs((vals * (dd ** 2).sum(1)).sum() * h * h - 2 * eps ** 2) < 1e-6 * eps ** 2 * 10


def test_walls_have_no_image(oracle_lib):
    G = 129
    h = 1.0 / (G - 1)
    w = _wl(2, False, 5 * h, G)
    p = oracle.params(w)
    sig, _ = oracle.deposit_kde(p, np.array([[0.0, 0.5]]), np.zeros(1, np.uint8))
    v = np.ones((G, G))
    v[0, :] *= 0.5; v[-1, :] *= 0.5; v[:, 0] *= 0.5; v[:, -1] *= 0.5
    mass = (sig.reshape(G, G) * v).sum() * h * h
    assert abs(mass - 0.5) < 1e-3


def test_step_uses_kernel_density_at_new_positions(oracle_lib):
    G, dt = 33, 1e-3
    h = 1.0 / G
    w = _wl(2, True, 2 * h, G, dt=dt, D_c=0.3, gamma=0.2,
            species=(W.Species(2 * h, 0.0, 0.0, 3.0, 0.0),))
    p = oracle.params(w)
    p.n_sub = 1
    c0 = np.linspace(0, 1, w.n_nodes)
    X0 = np.array([[0.3, 0.6]])
    X1, c1, _ = oracle.run(p, X0, np.zeros(1, np.uint8), c0, 0, 1)
    np.testing.assert_array_equal(X1, X0)  # D = 0, no drift, no forces
    sig, ups = oracle.deposit_kde(p, X1, np.zeros(1, np.uint8))
    np.testing.assert_allclose(c1, oracle.pde_density(p, c0, sig, ups), rtol=0, atol=0)
    # the PIC deposit gives a different field
    p.deposit_kernel = 0
    _, c2, _ = oracle.run(p, X0, np.zeros(1, np.uint8), c0, 0, 1)
    assert np.abs(c2 - c1).max() > 1e-4


def test_density_at_chosen_nodes_equals_the_full_grid(oracle_lib):
    """deposit_kde_at evaluates the same definition at chosen nodes: equal,
    bit for bit, to the full evaluation at every node of a small 3D case."""
    w = dataclasses.replace(W.scaled(W.workload(W.BLOBS_1M), n_agents=3000, grid_n=16),
                            deposit_kernel=1, kde_radius=3.0)
    inp = W.make_inputs(w)
    p = oracle.params(w)
    sig, ups = oracle.deposit_kde(p, inp["x0"], inp["species0"])
    nodes = np.random.default_rng(3).permutation(w.n_nodes)
    s2, u2 = oracle.deposit_kde_at(p, inp["x0"], inp["species0"], nodes)
    assert (sig > 0).sum() > 50
    assert np.array_equal(sig[nodes], s2) and np.array_equal(ups[nodes], u2)
