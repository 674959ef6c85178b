"""Pins of the oracle's type switching (eq. Chemo_reactions with the
fixed-step rule of Sect. 2.1: a reaction fires during [t, t + dt) when a
uniform draw falls below rate * dt).

* a two-type chain with constant rates a (0 -> 1) and b (1 -> 0): every agent
  is an independent two-state Markov chain with switching probabilities
  p = a dt and q = b dt per step, so the fraction of type 1 after n steps is
  pi* + (pi_0 - pi*)(1 - p - q)^n with pi* = p / (p + q), and the count is
  binomial;
* a concentration-dependent rate r_c c(X) with c(x, y) = x (linear, so its
  multilinear interpolation is exact): switch counts in bands of x match the
  sums of r_c x dt;
* the rate reads c^n at X^n, the position at the start of the step;
* the deposit of the step sees the new type;
* N_alpha + N_beta is conserved and a species without a reaction never
  changes.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _wl(species, n, periodic=True, grid_n=16, dt=1e-3, seed=91, D_c=0.0, gamma=0.0):
    return W.Workload("r", 2, periodic, 1.0, grid_n, dt, 0.0, D_c, gamma, 1, tuple(species),
                      (W.Instance(n, seed),))


def _sp(react_to=-1, rate=0.0, rate_c=0.0, chi=0.0, source=0.0, D=0.0):
    return W.Species(0.01, D, chi, source, 0.0, react_to, rate, rate_c)


def _binom_ok(count, n, prob, z=5.0):
    sd = math.sqrt(max(n * prob * (1 - prob), 1e-12))
    return abs(count - n * prob) < z * sd + 1


def test_two_type_chain_transient(oracle_lib):
    a, b, dt, n, steps = 20.0, 10.0, 1e-3, 60000, 25
    w = _wl([_sp(1, a), _sp(0, b)], n, dt=dt)
    p = oracle.params(w)
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, (n, 2))
    sp = (rng.uniform(size=n) < 0.3).astype(np.uint8)
    pi0 = sp.mean()
    c = np.zeros(w.n_nodes)
    P, Q = a * dt, b * dt
    pstar = P / (P + Q)
    st = 0
    for k in (1, 5, steps):
        while st < k:
            X, c, st, sp = oracle.step(p, X, sp, c, st, return_species=True)
        expect = pstar + (pi0 - pstar) * (1 - P - Q) ** k
        assert _binom_ok(int(sp.sum()), n, expect), (k, sp.mean(), expect)
    # the draws of different steps are independent: a one-step switch rate
    # of exactly p among the agents of type 0
    sp0 = sp.copy()
    _, _, _, sp1 = oracle.step(p, X, sp0, c, st, return_species=True)
    zero = sp0 == 0
    assert _binom_ok(int((sp1[zero] == 1).sum()), int(zero.sum()), P)


def test_concentration_dependent_rate_bands(oracle_lib):
    G, dt, rc, n = 17, 1e-3, 300.0, 200000
    w = _wl([_sp(), _sp(0, 0.0, rc)], n, periodic=False, grid_n=G, dt=dt)
    p = oracle.params(w)
    xs = W.node_coords(w)
    c = np.tile(xs, G)  # c(x, y) = x, x fastest
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 1, (n, 2))
    sp = np.ones(n, np.uint8)
    new = oracle.react(p, X, sp, c, 7)
    prob = rc * X[:, 0] * dt
    sw = new == 0
    for lo in np.arange(0, 1, 0.25):
        band = (X[:, 0] >= lo) & (X[:, 0] < lo + 0.25)
        mu = prob[band].sum()
        sd = math.sqrt((prob[band] * (1 - prob[band])).sum())
        assert abs(sw[band].sum() - mu) < 5 * sd + 1, (lo, sw[band].sum(), mu)
    # the same agents in y-bands: every band sees the mean rate rc * 0.5 * dt
    for lo in np.arange(0, 1, 0.25):
        band = (X[:, 1] >= lo) & (X[:, 1] < lo + 0.25)
        assert _binom_ok(int(sw[band].sum()), int(band.sum()), rc * 0.5 * dt, z=6)


@pytest.mark.parametrize("above", [False, True])
def test_rate_reads_concentration_at_start_of_step(above, oracle_lib):
    """One agent drifting up the gradient of c = x.  The threshold is set a
    hair below (or above) the agent's uniform at X^n; the drift would carry
    it far above the uniform at X^{n+1}."""
    G, dt, chi, seed = 17, 1e-3, 50.0, 1234
    x0 = np.array([[0.4, 0.3]])
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) ^ 0], np.uint32)
    w_ = oracle.philox(np.array([5, 0, 0, 1], np.uint32), key)[0]
    u = (((int(w_[0]) >> 8) | 1) / 2.0 ** 24)
    fac = (1 + 1e-6) if above else (1 - 1e-6)
    rc = u * fac / (x0[0, 0] * dt)
    w = _wl([_sp(), _sp(0, 0.0, rc, chi=chi)], 1, periodic=False, grid_n=G, dt=dt, seed=seed)
    p = oracle.params(w)
    c = np.tile(W.node_coords(w), G)
    X1, _, _, sp1 = oracle.run(p, x0, np.ones(1, np.uint8), c, 5, 1, return_species=True)
    assert X1[0, 0] > x0[0, 0] + 0.04  # the drift moved it well up the gradient
    assert int(sp1[0]) == (0 if above else 1)


def test_deposit_sees_the_new_type(oracle_lib):
    G, dt = 9, 1e-3
    x0 = np.array([[0.41, 0.57]])
    # type 0 (no source) switches with certainty (rate * dt = 1) to type 1 (source 3)
    w = _wl([_sp(1, 1.0 / dt), _sp(source=3.0)], 1, periodic=False, grid_n=G, dt=dt,
            D_c=0.2, gamma=0.1)
    p = oracle.params(w)
    c0 = np.linspace(0.0, 1.0, w.n_nodes)
    X1, c1, _, s1 = oracle.run(p, x0, np.zeros(1, np.uint8), c0, 0, 1, return_species=True)
    # the same step for an agent that is type 1 from the start
    w2 = _wl([_sp(), _sp(source=3.0)], 1, periodic=False, grid_n=G, dt=dt, D_c=0.2, gamma=0.1)
    X2, c2, _ = oracle.run(oracle.params(w2), x0, np.ones(1, np.uint8), c0, 0, 1)
    assert int(s1[0]) == 1
    np.testing.assert_array_equal(X1, X2)
    np.testing.assert_array_equal(c1, c2)
    # and without the switch the source term is absent
    w3 = _wl([_sp(), _sp(source=3.0)], 1, periodic=False, grid_n=G, dt=dt, D_c=0.2, gamma=0.1)
    _, c3, _ = oracle.run(oracle.params(w3), x0, np.zeros(1, np.uint8), c0, 0, 1)
    assert np.abs(c1 - c3).max() > 1e-3


def test_conservation_and_monotone_chain(oracle_lib):
    """0 -> 1 -> 2 with no way back: counts sum to N, no agent's type ever
    decreases, type 2 (no reaction) never changes."""
    n, dt = 20000, 1e-3
    w = _wl([_sp(1, 40.0, D=0.1), _sp(2, 0.0, 20.0, D=0.1), _sp(react_to=-1, rate=1e3, D=0.1)],
            n, dt=dt)
    p = oracle.params(w)
    rng = np.random.default_rng(5)
    X = rng.uniform(0, 1, (n, 2))
    sp = rng.integers(0, 3, n).astype(np.uint8)
    c = np.full(w.n_nodes, 2.0)
    st = 0
    for _ in range(12):
        prev = sp.copy()
        X, c, st, sp = oracle.step(p, X, sp, c, st, return_species=True)
        assert len(sp) == n and sp.max() <= 2
        assert np.all(sp >= prev)
        assert np.all(sp[prev == 2] == 2)
        assert np.all((sp - prev) <= 1)
    assert np.bincount(sp, minlength=3).sum() == n
    assert (sp == 2).sum() > (prev == 2).sum() - 1
