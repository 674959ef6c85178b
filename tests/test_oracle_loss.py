"""Pins of the oracle's density-mismatch loss (used to check the reverse mode).

* closed form: one agent on a node, zero target -> loss = (sum_k w_k^2)^dim;
* the smoothed histogram keeps total mass 1 and maps a constant to itself;
* the analytic position gradient matches central finite differences;
* FD of the loss in theta is smooth enough to have a plateau (sanity of the
  finite-difference reference used by the GPU adjoint tests);
* the float32 conditioning of the differentiation workload's segment
  derivatives: well inside 1e-3 over one step, percents over 20.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _taps(sigma):
    R = math.floor(3 * sigma + 0.5)
    w = np.exp(-0.5 * np.arange(-R, R + 1) ** 2 / sigma**2)
    return w / w.sum()


@pytest.mark.parametrize("dim", [2, 3])
def test_single_agent_on_node_closed_form(dim, oracle_lib):
    m = 16
    X = np.full((1, dim), 5.0 / m)
    loss = oracle.density_loss(dim, 1.0, X, np.zeros(m ** dim), m, 1.5)
    assert abs(loss - (np.sum(_taps(1.5) ** 2)) ** dim) < 1e-14


def test_mass_and_constant_target(oracle_lib):
    m, n = 32, 2000
    X = np.random.default_rng(3).uniform(0, 1, (n, 2))
    # target = uniform density 1/m^2 everywhere: loss = sum (rho_s - 1/H)^2 and
    # sum(rho_s) = 1 means mean(rho_s - 1/H) = 0
    H = m * m
    loss, g = oracle.density_loss(2, 1.0, X, np.full(H, 1.0 / H), m, 2.0, grad=True)
    assert loss > 0
    # moving every agent by the same shift leaves the histogram's mass
    # unchanged: the gradient summed over agents of a uniform target is the
    # derivative of a translation, small but the mass pin is exact:
    loss0 = oracle.density_loss(2, 1.0, X, np.zeros(H), m, 2.0)
    # with zero target the loss is sum rho_s^2 >= (sum rho_s)^2 / H = 1 / H
    assert loss0 >= 1.0 / H - 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_matches_finite_differences(dim, oracle_lib):
    m, n = 12, 300
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 1, (n, dim))
    target = rng.uniform(0, 2.0 / m ** dim, m ** dim)
    loss, g = oracle.density_loss(dim, 1.0, X, target, m, 1.3, grad=True)
    h = 1e-7
    for i in rng.integers(0, n, 12):
        for a in range(dim):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, a] += h
            Xm[i, a] -= h
            fd = (oracle.density_loss(dim, 1.0, Xp, target, m, 1.3) -
                  oracle.density_loss(dim, 1.0, Xm, target, m, 1.3)) / (2 * h)
            assert abs(fd - g[i, a]) <= 1e-6 * max(1.0, abs(g).max())


def test_hist_matches_loss_definition(oracle_lib):
    m, n = 20, 700
    X = np.random.default_rng(5).uniform(0, 1, (n, 2))
    rho = oracle.density_hist(2, 1.0, X, m, 2.0)
    assert abs(rho.sum() - 1.0) < 1e-12          # smoothing keeps the mass
    t = np.random.default_rng(6).uniform(0, 2e-3, m * m)
    assert abs(oracle.density_loss(2, 1.0, X, t, m, 2.0) - ((rho - t) ** 2).sum()) < 1e-15


def test_theta_finite_differences_have_a_plateau(oracle_lib):
    """Central differences of loss(theta) agree across step sizes, so the FD
    reference of the reverse-mode tests is well defined."""
    w = W.scaled(W.adjoint_2d(), n_agents=1500, grid_n=32, steps=10)
    inp = W.make_inputs(w)
    tw = W.scaled(W.adjoint_2d(chi=1.5, k=800, D=0.8, seed=2005), n_agents=1500, grid_n=32)
    m = 16
    target = oracle.target_hist(tw, W.make_inputs(tw), 10, m, 2.0)
    theta = np.array([1.0, 100.0, 1.0])
    base = oracle.loss_at(w, inp, theta, target, 10, m, 2.0)
    assert base > 0
    for j in range(3):
        fds = []
        for rel in (1e-3, 1e-4):
            h = rel * theta[j]
            tp, tm = theta.copy(), theta.copy()
            tp[j] += h
            tm[j] -= h
            fds.append((oracle.loss_at(w, inp, tp, target, 10, m, 2.0) -
                        oracle.loss_at(w, inp, tm, target, 10, m, 2.0)) / (2 * h))
        scale = max(abs(fds[0]), 1e-12)
        assert abs(fds[0] - fds[1]) <= 2e-2 * scale + 1e-10


def test_differentiation_segment_derivatives_float32_conditioning():
    """Why the reverse-mode gate of a 20-step segment of the differentiation
    workload carries the derivative's own float32 conditioning.  On the
    oracle alone, the scale derivatives (chi, k, D) of three linear
    functionals (displacements with random weights, the field with random
    node weights, a smooth field moment) are compared along the FP64
    trajectory and along trajectories perturbed by half a float32 ulp per
    step: over one step they agree far inside the 1e-3 bar, over 20 steps
    some differ by more than 1e-2."""
    from adjoint_ref import segment_fd_ensemble
    w = W.adjoint_2d()
    inp = W.make_inputs(w)
    rng = np.random.default_rng(4000)
    wX = rng.standard_normal((w.n_total, 2))
    wC = rng.standard_normal(w.n_nodes)
    xs = W.node_coords(w)
    gx, gy = np.meshgrid(xs, xs, indexing="xy")
    wS = (np.sin(2 * np.pi * gx) * np.cos(2 * np.pi * gy)).reshape(-1)
    x64 = inp["x0"].astype(np.float64)

    def funcs(X, c):
        d = X - x64
        d -= np.rint(d)
        return [float((wX * d).sum()), float((wC * c).sum()), float((wS * c).sum())]

    theta = np.array([1.0, 100.0, 1.0])
    worst = {}
    for K in (1, 20):
        fd0, mem = segment_fd_ensemble(w, inp["x0"], inp["species0"], inp["c0"], 0, K, theta,
                                       funcs, M=2, seed=7)
        sig = np.sqrt(((mem - fd0) ** 2).mean(0))
        nz = np.abs(fd0) > 0
        worst[K] = float((sig[nz] / np.abs(fd0[nz])).max())
    print(f"float32 conditioning, worst of 9: 1 step {worst[1]:.1e}, 20 steps {worst[20]:.1e}")
    assert worst[1] < 2e-4
    assert worst[20] > 1e-2
