"""Gaussian kernel density deposit on the GPU against the FP64 oracle,
through the C ABI: the agent-side scatter (LDS table, then float atomics;
the default in 3D) and the per-node gather over the cell list of X^{n+1}
(fixed order; 2D, and deterministic mode).

Bars: positions as the plain step (1e-5 L per step).  The field after a
step lies within 1e-5 max|c| of the oracle's field bracketed by truncation
radii kde_radius (1 -/+ 1e-5): a node-agent pair at the truncation radius
may be decided either way in float32.  In deterministic mode graph replay
equals eager replay bit for bit and runs repeat bit for bit.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import make_sim, pos_err

pytestmark = pytest.mark.gpu


def _kde(w, kappa=3.0):
    return dataclasses.replace(w, deposit_kernel=1, kde_radius=kappa)


def _case(name, n, g, kappa=3.0):
    if name == W.ENSEMBLE_256:
        w = W.scaled(W.workload(W.ENSEMBLE_256),
                     n_agents=list(np.random.default_rng(9).integers(1, 900, 6)), grid_n=g)
    else:
        w = W.scaled(W.workload(name), n_agents=n, grid_n=g)
    return _kde(w, kappa)


def _bracket(w, inp, steps):
    lo = oracle.run_workload(dataclasses.replace(w, kde_radius=w.kde_radius * (1 - 1e-5)), inp,
                             steps)
    hi = oracle.run_workload(dataclasses.replace(w, kde_radius=w.kde_radius * (1 + 1e-5)), inp,
                             steps)
    return lo, hi


def _within(c, lo, hi, tol):
    a, b = np.minimum(lo, hi), np.maximum(lo, hi)
    return np.all(c >= a - tol) and np.all(c <= b + tol)


CASES = [(W.PERIODIC_1K, 3001, 37, 3.0), (W.WALLS_100K, 20011, 129, 3.0),
         (W.BLOBS_1M, 8000, 32, 3.0), (W.ADJOINT_50K, 6000, 48, 3.0),
         (W.ENSEMBLE_256, None, 24, 3.0), (W.PERIODIC_1K, 3001, 37, 1.5),
         (W.WALLS_100K, 5000, 65, 6.0),
         # 33^3 nodes: the last work-group of the 3D gather is ragged
         (W.BLOBS_1M, 6007, 33, 3.0)]


@pytest.mark.parametrize("det", [False, True], ids=["scatter", "gather"])
@pytest.mark.parametrize("name,n,g,kappa", CASES)
def test_one_step_matches_oracle(name, n, g, kappa, det):
    """Both forms of the deposit in 3D: the agent-side scatter (float
    atomics) and, where results must repeat bit for bit, the fixed-order
    gather (the 2D cases run the gather either way)."""
    w = _case(name, n, g, kappa)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp, deterministic=det)
    assert sim.info["deposit_path"] == 4
    sim.step(1)
    x, c, _ = sim.get_state()
    (Xlo, clo), (Xhi, chi_) = _bracket(w, inp, 1)
    assert pos_err(x.cpu().numpy(), Xlo, w.L, w.periodic) <= 1e-5
    scale = max(np.abs(clo).max(), 1e-30)
    assert _within(c.cpu().numpy().astype(np.float64), clo, chi_, 1e-5 * scale)


def _w3(n, g, periodic, species, kappa, rule="halves", seed=1203):
    return W.Workload("kde3d", 3, periodic, 1.0, g, 1e-6, 100.0, 1.0, 0.1, 1, tuple(species),
                      (W.Instance(n, seed),), species_rule=rule,
                      c0="sin" if periodic else "cos", gen_seed=seed, deposit_kernel=1,
                      kde_radius=kappa)


# 3D agent-side scatter at the ball sizes of the full workload (radius about
# 1.5 to 3 node spacings, so every agent walks a box of several nodes per
# axis, across the periodic seam), with two species of different radii and
# uptake, with walls, with kappa = 6, and with uniform agents whose
# 1024-agent work-groups reach far more than the 4096 slots of the LDS table
# (the overflow goes to device atomics).
SCATTER_3D = {
    "wide_balls_torus": _w3(6000, 32, True, [W.Species(0.02, 1.0, 1.0, 1.0, 0.0)], 3.0,
                            rule="single"),
    "two_species_uptake_walls": _w3(6000, 33, False, [W.Species(0.015, 1.0, 0.0, 1.0, 0.0),
                                                      W.Species(0.025, 0.5, 2.0, 0.0, 1.0)],
                                    3.0),
    "kappa6_two_species_torus": _w3(4000, 32, True, [W.Species(0.01, 1.0, 0.0, 1.0, 0.0),
                                                     W.Species(0.015, 0.5, 1.0, 0.5, 2.0)],
                                    6.0),
    "lds_table_overflow": _w3(16000, 40, True, [W.Species(0.025, 1.0, 1.0, 1.0, 0.0)], 3.0,
                              rule="single"),
}


def _nodes_per_workgroup(w, x):
    """Distinct nodes inside the balls of each 1024-agent run of the
    cell-sorted order (the scatter's work-groups), counted on the host."""
    d = max(s.diameter for s in w.species)
    nb = int(np.floor(w.L / (d * (1 + 1e-4))))
    b = np.minimum((x * nb / w.L).astype(np.int64), nb - 1)
    order = np.argsort(b[:, 0] + nb * (b[:, 1] + nb * b[:, 2]), kind="stable")
    n = w.grid_n
    h = w.L / n if w.periodic else w.L / (n - 1)
    R = w.kde_radius * d
    r = int(np.ceil(R / h))
    off = np.stack(np.meshgrid(*([np.arange(-r, r + 1)] * 3), indexing="ij"), -1).reshape(-1, 3)
    out = []
    for g0 in range(0, len(order), 1024):
        xs = x[order[g0:g0 + 1024]].astype(np.float64)
        base = np.floor(xs / h).astype(np.int64)
        cand = (base[:, None, :] + off[None, :, :])
        dist2 = ((cand * h - xs[:, None, :]) ** 2).sum(-1)
        keep = cand[dist2 < R * R] % n
        out.append(len(np.unique(keep[:, 0] + n * (keep[:, 1] + n * keep[:, 2]))))
    return out


@pytest.mark.parametrize("case", sorted(SCATTER_3D))
def test_one_step_3d_scatter_cases(case):
    w = SCATTER_3D[case]
    inp = W.make_inputs(w)
    if case == "lds_table_overflow":
        assert max(_nodes_per_workgroup(w, inp["x0"])) > 2 * 4096
    sim = make_sim(w, inp)
    assert sim.info["deposit_path"] == 4
    sim.step(1)
    x, c, _ = sim.get_state()
    (Xlo, clo), (Xhi, chi_) = _bracket(w, inp, 1)
    assert pos_err(x.cpu().numpy(), Xlo, w.L, w.periodic) <= 1e-5
    scale = max(np.abs(clo).max(), 1e-30)
    cg = c.cpu().numpy().astype(np.float64)
    print(f"{case}: field dev from bracket {max((np.minimum(clo, chi_) - cg).max(), (cg - np.maximum(clo, chi_)).max(), 0.0) / scale:.2e}")
    assert _within(cg, clo, chi_, 1e-5 * scale)
    # a second step: the pairs cleared by the last PDE substep start at zero
    sim.step(1)
    x2, c2, _ = sim.get_state()
    here = dict(inp, x0=x.cpu().numpy(), c0=c.cpu().numpy())
    lo2 = oracle.run_workload(dataclasses.replace(w, kde_radius=w.kde_radius * (1 - 1e-5)),
                              here, 1, step0=1)
    hi2 = oracle.run_workload(dataclasses.replace(w, kde_radius=w.kde_radius * (1 + 1e-5)),
                              here, 1, step0=1)
    assert pos_err(x2.cpu().numpy(), lo2[0], w.L, w.periodic) <= 1e-5
    scale2 = max(np.abs(lo2[1]).max(), 1e-30)
    assert _within(c2.cpu().numpy().astype(np.float64), lo2[1], hi2[1], 1e-5 * scale2)


def test_one_step_full_size_walls_100k():
    """The full 100k walls workload with the kernel density deposit as the
    benchmark runs it (radius 3 bandwidths, default launch)."""
    w = _kde(W.workload(W.WALLS_100K), 3.0)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.step(1)
    x, c, _ = sim.get_state()
    (Xlo, clo), (Xhi, chi_) = _bracket(w, inp, 1)
    assert pos_err(x.cpu().numpy(), Xlo, w.L, w.periodic) <= 1e-5
    scale = max(np.abs(clo).max(), 1e-30)
    assert _within(c.cpu().numpy().astype(np.float64), clo, chi_, 1e-5 * scale)


def test_one_step_full_size_3d_sampled_nodes():
    """The full 1M-agent 3D workload with the kernel density deposit as the
    benchmark runs it.  The oracle's density is a sum over every agent at
    every node (2e12 terms here), so it is taken at 400 nodes: 300 at the
    cells of random agents and 100 anywhere, from the device's own new
    positions (in the blob cores a 1e-7 position difference would move the
    density by more than the bar).  With one PDE substep a node's new value
    needs only its own density and the old field, so the oracle's PDE with
    the densities of the other nodes zeroed is exact at those nodes.
    Positions: the oracle's step with the particle-in-cell deposit (the
    update does not depend on the deposit kernel)."""
    w = _kde(W.workload(W.BLOBS_1M), 3.0)
    inp = W.make_inputs(w)
    p = oracle.params(w)
    assert p.n_sub == 1
    sim = make_sim(w, inp)
    sim.step(1)
    x, c, _ = sim.get_state()
    x, c = x.cpu().numpy(), c.cpu().numpy()
    Xo, _ = oracle.run_workload(dataclasses.replace(w, deposit_kernel=0), inp, 1)
    assert pos_err(x, Xo, w.L, w.periodic) <= 1e-5
    rng = np.random.default_rng(11)
    n = w.grid_n
    cells = np.floor(Xo[rng.integers(0, w.n_total, 300)] * n).astype(np.int64) % n
    nodes = np.unique(np.concatenate([cells[:, 0] + n * cells[:, 1] + n * n * cells[:, 2],
                                      rng.integers(0, w.n_nodes, 100)]))
    refs = []
    for kappa in (3.0 * (1 - 1e-5), 3.0 * (1 + 1e-5)):
        pk = oracle.params(dataclasses.replace(w, kde_radius=kappa))
        sig, ups = oracle.deposit_kde_at(pk, x.astype(np.float64), inp["species0"], nodes)
        sf, uf = np.zeros(w.n_nodes), np.zeros(w.n_nodes)
        sf[nodes], uf[nodes] = sig, ups
        refs.append(oracle.pde_density(pk, inp["c0"], sf, uf)[nodes])
        assert (sig > 0).sum() >= 250
    scale = max(np.abs(refs[0]).max(), np.abs(inp["c0"]).max())
    assert _within(c[nodes].astype(np.float64), refs[0], refs[1], 1e-5 * scale)


def test_one_step_3d_batched_instances():
    """Three 3D instances in one batch (17^3 nodes each, ragged in total):
    every node's gather stays inside its own instance's cell list."""
    w = _kde(W.scaled(W.workload(W.BLOBS_1M), n_agents=[1500, 2003, 700], grid_n=17))
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.step(1)
    x, c, _ = sim.get_state()
    (Xlo, clo), (Xhi, chi_) = _bracket(w, inp, 1)
    assert pos_err(x.cpu().numpy(), Xlo, w.L, w.periodic) <= 1e-5
    scale = max(np.abs(clo).max(), 1e-30)
    assert _within(c.cpu().numpy().astype(np.float64), clo, chi_, 1e-5 * scale)
    assert np.abs(clo).max() > 0


@pytest.mark.parametrize("name,n,g,steps", [(W.PERIODIC_1K, 2000, 37, 10),
                                            (W.WALLS_100K, 8000, 65, 6),
                                            (W.BLOBS_1M, 4000, 33, 4)])
def test_trajectory_matches_oracle(name, n, g, steps):
    w = _case(name, n, g)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.use_graph(True)
    sim.step(steps)
    x, c, _ = sim.get_state()
    (Xlo, clo), (Xhi, chi_) = _bracket(w, inp, steps)
    assert pos_err(x.cpu().numpy(), Xlo, w.L, w.periodic) <= 1e-5 * steps
    scale = max(np.abs(clo).max(), 1e-30)
    assert _within(c.cpu().numpy().astype(np.float64), clo, chi_, 1e-5 * steps * scale)


@pytest.mark.parametrize("name,n,g", [(W.WALLS_100K, 6000, 65), (W.BLOBS_1M, 6007, 33)])
def test_graph_equals_eager_and_deterministic_repeats(name, n, g):
    """3D: the split row walk sums its partials in a fixed order."""
    w = _case(name, n, g)
    inp = W.make_inputs(w)
    runs = []
    for graph in (False, True, True):
        sim = make_sim(w, inp, deterministic=True)
        sim.use_graph(graph)
        sim.step(9)
        sim.sync()
        x, c, st = sim.get_state()
        assert st == 9
        runs.append((x.cpu().numpy(), c.cpu().numpy()))
        sim.close()
    for x, c in runs[1:]:
        assert np.array_equal(x, runs[0][0]) and np.array_equal(c, runs[0][1])


def test_profile_and_set_state_round_trip():
    import torch
    w = _case(W.PERIODIC_1K, 3000, 37)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    prof = sim.profile_steps(3)
    assert prof["deposit"] > 0 and prof["pde"] > 0 and prof["update"] > 0
    sim.set_state(torch.from_numpy(inp["x0"]), torch.from_numpy(inp["c0"]), 0)
    sim.step(1)
    x, c, _ = sim.get_state()
    (Xlo, clo), (_, chi_) = _bracket(w, inp, 1)
    assert pos_err(x.cpu().numpy(), Xlo, w.L, w.periodic) <= 1e-5
    assert _within(c.cpu().numpy().astype(np.float64), clo, chi_, 1e-5 * np.abs(clo).max())


def test_rejections():
    import torch
    from paper_1805_11007_amd import PcError
    w = _case(W.ADJOINT_50K, 2000, 32)
    inp = W.make_inputs(w)
    with pytest.raises(PcError):
        make_sim(w, inp, deposit_mode=3)
    with pytest.raises(PcError):
        make_sim(w, inp, kde_radius=60.0)   # 60 * 0.01 >= L / 2
    sim = make_sim(w, inp, adjoint_steps=2)
    with pytest.raises(PcError):
        sim.adjoint_segment(torch.zeros(w.n_total, 2), torch.zeros(w.n_nodes), 1)
