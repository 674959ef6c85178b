"""Pair and update variants on the GPU against the FP64 oracle, through the
C ABI: the exponential potential (Sect. 4) with its range cut, tamed Euler
(eq. sde_ETamed) and the hard-sphere overlap correction (Sect. 2.2).

Bars: neighbour sets bit-exact (decided in float32 on both sides, the
exponential's range included); forces within 1e-5 of the force scale;
positions within 1e-5 L per step (the overlap correction is continuous at
contact, so float32 rounding of a near-contact decision moves nothing);
field within 1e-5 max|c| per step; graph replay and deterministic mode
bit for bit.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import (field_err, field_from_positions, field_ok, make_sim, oracle_forces,
                         pos_err)

pytestmark = pytest.mark.gpu


def _v(name, n, g, **kw):
    return dataclasses.replace(W.scaled(W.workload(name), n_agents=n, grid_n=g), **kw)


def _oracle_nbrs_scaled(w, inp, scale):
    diam = [s.diameter * scale for s in w.species]
    cnt, hs = oracle.neighbours_f32(w.dim, w.periodic, w.L, inp["x0"], inp["species0"],
                                    np.arange(w.n_total, dtype=np.uint32), diam)
    return cnt, hs


@pytest.mark.parametrize("name,n,g", [(W.PERIODIC_1K, 3001, 37), (W.WALLS_100K, 20011, 129), (W.BLOBS_1M, 20000, 32)])
def test_exponential_neighbours_and_forces(name, n, g):
    w = _v(name, n, g, potential=1, pot_range=2.5, k=5.0)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    cnt, hsh = sim.debug_neighbours()
    ocnt, ohsh = _oracle_nbrs_scaled(w, inp, 2.5)
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ocnt)
    assert np.array_equal(hsh.cpu().numpy().view(np.uint64), ohsh)
    F = sim.debug_forces().cpu().numpy().astype(np.float64)
    Fo = oracle_forces(w, inp)
    scale = w.k / min(s.diameter for s in w.species)
    assert np.abs(F - Fo).max() <= 1e-5 * scale


CASES = [
    (W.PERIODIC_1K, 3001, 37, dict(potential=1, pot_range=3.0, k=2.0)),
    (W.WALLS_100K, 20011, 129, dict(potential=1, pot_range=2.0, k=0.5)),
    (W.PERIODIC_1K, 3001, 37, dict(potential=0, tamed=True, k=1e5)),
    (W.BLOBS_1M, 20000, 32, dict(potential=0, tamed=True, k=1e6)),
    (W.PERIODIC_1K, 3001, 37, dict(potential=2)),
    (W.WALLS_100K, 20011, 129, dict(potential=2)),
    (W.BLOBS_1M, 20000, 32, dict(potential=2)),
    (W.ADJOINT_50K, 6000, 48, dict(potential=2)),
]


@pytest.mark.parametrize("name,n,g,kw", CASES)
def test_one_step(name, n, g, kw):
    w = _v(name, n, g, **kw)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.step(1)
    x, c, _ = sim.get_state()
    Xo, co = oracle.run_workload(w, inp, 1)
    assert pos_err(x.cpu().numpy(), Xo, w.L, w.periodic) <= 1e-5
    assert field_err(c.cpu().numpy(), co) <= 1e-5


@pytest.mark.parametrize("name", [W.WALLS_100K, W.BLOBS_1M])
@pytest.mark.parametrize("kw", [dict(potential=1, pot_range=3.0, k=1.0), dict(tamed=True),
                                dict(potential=2)], ids=["exponential", "tamed", "hard_spheres"])
def test_one_step_full_size(name, kw):
    """The full 100k walls and 1M 3D workloads with each variant as the
    benchmark runs it (default launch).  Positions against the oracle's
    step (1e-5 L).  Exponential and tamed: the field against the oracle's
    step and against its deposit and PDE at the device's own new positions
    (1e-5 max|c|).  Hard spheres: the correction maps a near-coincident
    pair's distance r to 2d - r, so a rounding difference in r moves both
    agents, and on the 512^2 grid one agent's deposit weighs enough for such
    a move (inside the position bar) to show in the field; its field is
    compared at the device's own positions, within 1e-5 max|c| plus the
    float32 rounding bound of the deposit weights."""
    w = dataclasses.replace(W.workload(name), **kw)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.step(1)
    x, c, _ = sim.get_state()
    x, c = x.cpu().numpy(), c.cpu().numpy()
    Xo, co = oracle.run_workload(w, inp, 1)
    ex = pos_err(x, Xo, w.L, w.periodic)
    c_ref = field_from_positions(w, inp["c0"], x, inp["species0"])
    ec, ecp = field_err(c, co), field_err(c, c_ref)
    print(f"{name} {kw}: position err {ex:.2e} field err {ec:.2e} "
          f"(at device positions {ecp:.2e})")
    assert ex <= 1e-5
    if kw.get("potential") == 2:
        assert field_ok(c, c_ref, w, x, inp["species0"])
    else:
        assert ec <= 1e-5
        assert ecp <= 1e-5


@pytest.mark.parametrize("name,n,g,kw,steps", [
    (W.PERIODIC_1K, 2000, 37, dict(potential=2), 10),
    (W.WALLS_100K, 8000, 65, dict(potential=2), 8),
    (W.PERIODIC_1K, 2000, 37, dict(potential=1, pot_range=3.0, k=2.0), 10),
    (W.PERIODIC_1K, 2000, 37, dict(potential=0, tamed=True, k=1e5), 10),
])
def test_trajectory(name, n, g, kw, steps):
    """Soft potentials at moderate stiffness: the whole trajectory within
    1e-5 per step.  Hard spheres: the overlap correction maps a pair's
    distance r to 2d - r, and clusters of overlaps pass a rounding
    difference on to every member, so trajectories of the two precisions
    separate faster than linearly.  The tamed harmonic step at k dt = 1 is
    as stiff: an overlapping pair's separation update has a Jacobian of
    order one, so a float32 rounding (~1e-7 L per step) grows about a
    thousandfold in 10 steps.  For both, every step is checked from the
    GPU's own state instead (1e-5), and the whole trajectory within 1e-3."""
    w = _v(name, n, g, **kw)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    if kw.get("potential") == 2 or kw.get("tamed"):
        for t in range(steps):
            x, c, st = sim.get_state()
            assert st == t
            sim.step(1)
            x1, c1, _ = sim.get_state()
            here = {"x0": x.cpu().numpy(), "species0": inp["species0"], "c0": c.cpu().numpy()}
            Xo, co = oracle.run_workload(w, here, 1, step0=t)
            assert pos_err(x1.cpu().numpy(), Xo, w.L, w.periodic) <= 1e-5, t
            assert field_err(c1.cpu().numpy(), co) <= 1e-5, t
        Xo, co = oracle.run_workload(w, inp, steps)
        assert pos_err(x1.cpu().numpy(), Xo, w.L, w.periodic) <= 1e-3
        return
    sim.use_graph(True)
    sim.step(steps)
    x, c, _ = sim.get_state()
    Xo, co = oracle.run_workload(w, inp, steps)
    assert pos_err(x.cpu().numpy(), Xo, w.L, w.periodic) <= 1e-5 * steps
    assert field_err(c.cpu().numpy(), co) <= 1e-5 * steps


def test_hard_spheres_reduce_overlap_and_repeat_bitwise():
    w = _v(W.PERIODIC_1K, 4000, 37, potential=2)
    inp = W.make_inputs(w)
    runs = []
    for graph in (False, True):
        sim = make_sim(w, inp, deterministic=True)
        sim.use_graph(graph)
        sim.step(11)
        x, c, _ = sim.get_state()
        runs.append((x.cpu().numpy(), c.cpu().numpy()))
        prof = sim.profile_steps(2)
        assert prof["overlap"] > 0
        sim.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    from scipy.spatial import cKDTree
    d = w.species[0].diameter

    def overlap(X):
        pr = cKDTree(X, boxsize=1.0).query_pairs(d, output_type="ndarray")
        dx = X[pr[:, 1]] - X[pr[:, 0]]
        dx -= np.rint(dx)
        return (d - np.sqrt((dx ** 2).sum(1))).sum()

    assert overlap(runs[0][0].astype(np.float64)) < 0.5 * overlap(inp["x0"].astype(np.float64))


def test_rejections():
    import torch
    from paper_1805_11007_amd import PcError
    w = _v(W.ADJOINT_50K, 2000, 32, potential=2, deposit_kernel=1)
    with pytest.raises(PcError):
        make_sim(w, W.make_inputs(w))
    w = _v(W.ADJOINT_50K, 2000, 32, potential=1, pot_range=0.5)
    with pytest.raises(PcError):
        make_sim(w, W.make_inputs(w))
    w = _v(W.ADJOINT_50K, 2000, 32, potential=1)
    sim = make_sim(w, W.make_inputs(w), adjoint_steps=2)
    with pytest.raises(PcError):
        sim.adjoint_segment(torch.zeros(w.n_total, 2), torch.zeros(w.n_nodes), 1)
