"""GPU library vs FP64 oracle, element by element, through the C ABI.

Bars: neighbour sets bit-exact (counts and id hashes decided in float32 on
both sides); positions within 1e-5 of L per step (minimum image);
the chemical within 1e-5 of max|c| per step; forces within float32
accumulation error of the force scale k * d.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import (field_err, field_from_positions, make_sim, oracle_forces,
                         oracle_neighbours, oracle_steps, pos_err)

pytestmark = pytest.mark.gpu

# (workload, agents, grid) cases: several bins / tiles with ragged tails
SMALL = [(W.PERIODIC_1K, 1000, None), (W.PERIODIC_1K, 3001, 37), (W.WALLS_100K, 20011, 129),
         (W.BLOBS_1M, 40000, 48), (W.ENSEMBLE_256, None, 32), (W.ADJOINT_50K, 9000, 64)]
FULL = [W.PERIODIC_1K, W.WALLS_100K, W.BLOBS_1M, W.ADJOINT_50K]


def _w(name, n, g):
    w = W.workload(name)
    if name == W.ENSEMBLE_256:
        rng = np.random.default_rng(4)
        sizes = list(rng.integers(1, 900, 12)) + [1, 2]
        return W.scaled(w, n_agents=sizes, grid_n=g)
    return W.scaled(w, n_agents=n, grid_n=g)


@pytest.mark.parametrize("name,n,g", SMALL)
def test_neighbour_sets_bit_exact(name, n, g):
    w = _w(name, n, g)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    cnt, hsh = sim.debug_neighbours()
    ocnt, ohsh = oracle_neighbours(w, inp)
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ocnt)
    assert np.array_equal(hsh.cpu().numpy().view(np.uint64), ohsh)


@pytest.mark.parametrize("name", FULL)
def test_neighbour_sets_bit_exact_full_size(name):
    w = W.workload(name)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    cnt, hsh = sim.debug_neighbours()
    ocnt, ohsh = oracle_neighbours(w, inp)
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ocnt)
    assert np.array_equal(hsh.cpu().numpy().view(np.uint64), ohsh)


@pytest.mark.parametrize("det", [False, True])
def test_pair_walk_after_lds_hash_deposits(det):
    """3D, after steps with the LDS-hash deposit, whose table is filled with
    0xFFFFFFFF: outside deterministic mode a lane walks its stencil rows
    longest first from an LDS table of row starts, which every row must
    write (a stale slot would wrap the walk).  Neighbour sets bit-exact and
    forces against the oracle at the device's own positions; the debug
    kernel walks the rows as the update does.  Forces are compared away
    from the periodic seam (the agents the sorted walk serves): across it,
    x_j - x_i of coordinates near 0 and near L rounds to an ulp of L before
    the shift, which a close pair's factor k (d / r - 1) multiplies (8e-5
    at r = d / 4, whatever the row order)."""
    w = W.scaled(W.workload(W.BLOBS_1M), n_agents=250000, grid_n=40)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp, deterministic=det, deposit_mode=1)
    sim.step(3)
    sim.sync()
    here = {"x0": sim.positions().cpu().numpy(), "species0": inp["species0"]}
    cnt, hsh = sim.debug_neighbours()
    ocnt, ohsh = oracle_neighbours(w, here)
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ocnt)
    assert np.array_equal(hsh.cpu().numpy().view(np.uint64), ohsh)
    assert ocnt.mean() > 1.0   # 1.5 neighbours per agent at a quarter of the agents
    F = sim.debug_forces().cpu().numpy().astype(np.float64)
    Fo = oracle_forces(w, here)
    d = max(s.diameter for s in w.species)
    inner = np.all((here["x0"] >= 2 * d) & (here["x0"] <= w.L - 2 * d), axis=1)
    assert inner.mean() > 0.9
    assert np.abs(F - Fo)[inner].max() <= 1e-5 * w.k * d


def test_pair_walk_rows_beyond_2047_agents():
    """3D pile: 30,000 of 36,000 agents inside 3 x 3 x 3 bins (~1,100 each),
    so stencil rows hold more agents than the 16-bit keys of the
    longest-row-first walk carry (2047); waves with such a row take the
    fixed-order walk.  Neighbour sets bit-exact and forces against the
    oracle (non-deterministic mode)."""
    w = W.scaled(W.workload(W.BLOBS_1M), n_agents=36000, grid_n=32)
    inp = W.make_inputs(w)
    x0 = inp["x0"].copy()
    rng = np.random.default_rng(7)
    lo, side = 125 / 249 + 1e-6, 3 / 249 - 2e-6   # bins 125..127 of 249 on each axis
    x0[:30000] = (lo + rng.uniform(0, side, (30000, 3))).astype(np.float32)
    inp = dict(inp, x0=x0)
    sim = make_sim(w, inp)
    cnt, hsh = sim.debug_neighbours()
    ocnt, ohsh = oracle_neighbours(w, inp)
    assert ocnt.max() > 2047
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ocnt)
    assert np.array_equal(hsh.cpu().numpy().view(np.uint64), ohsh)
    F = sim.debug_forces().cpu().numpy().astype(np.float64)
    Fo = oracle_forces(w, inp)
    # a pile agent sums up to ~4,700 float32 pair terms of size up to k d:
    # 1e-5 k d plus 2^-19 k d per neighbour (a float32 emulation of the same
    # sums on the CPU reaches 0.17 of it)
    kd = w.k * max(s.diameter for s in w.species)
    bar = 1e-5 * kd + 2.0 ** -19 * kd * ocnt.astype(np.float64)
    assert np.all(np.abs(F - Fo).max(axis=1) <= bar)


def test_pair_walk_rows_beyond_2047_agents_2d():
    """2D pile: 12,000 of 14,000 agents inside 3 x 3 bins (~1,330 each), so
    the three-bin rows of the longest-row-first walk exceed its 2047-agent
    keys and those waves take the fixed-order walk.  Neighbour sets
    bit-exact and forces against the oracle (non-deterministic mode)."""
    w = W.scaled(W.workload(W.PERIODIC_1K), n_agents=14000, grid_n=64)
    inp = W.make_inputs(w)
    nb = int(np.floor(w.L / (max(s.diameter for s in w.species) * (1 + 1e-4))))
    x0 = inp["x0"].copy()
    rng = np.random.default_rng(9)
    lo, side = (nb // 2) / nb + 1e-6, 3 / nb - 2e-6   # bins nb/2 .. nb/2 + 2 on both axes
    x0[:12000] = (lo + rng.uniform(0, side, (12000, 2))).astype(np.float32)
    inp = dict(inp, x0=x0)
    sim = make_sim(w, inp)
    cnt, hsh = sim.debug_neighbours()
    ocnt, ohsh = oracle_neighbours(w, inp)
    assert ocnt.max() > 2047
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ocnt)
    assert np.array_equal(hsh.cpu().numpy().view(np.uint64), ohsh)
    F = sim.debug_forces().cpu().numpy().astype(np.float64)
    Fo = oracle_forces(w, inp)
    d = max(s.diameter for s in w.species)
    kd = w.k * d
    # as in 3D: 1e-5 k d plus 2^-19 k d per neighbour (the float32 emulation
    # reaches 0.31 of it here)
    bar = 1e-5 * kd + 2.0 ** -19 * kd * ocnt.astype(np.float64)
    # off the periodic seam, where x_j - x_i rounds to an ulp of L
    inner = np.all((x0 >= 2 * d) & (x0 <= w.L - 2 * d), axis=1)
    assert np.all(np.abs(F - Fo).max(axis=1)[inner] <= bar[inner])


@pytest.mark.parametrize("name,n,g", SMALL)
def test_forces(name, n, g):
    w = _w(name, n, g)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    F = sim.debug_forces().cpu().numpy().astype(np.float64)
    Fo = oracle_forces(w, inp)
    scale = w.k * max(s.diameter for s in w.species)
    assert np.abs(F - Fo).max() <= 1e-5 * scale
    assert np.abs(F.sum(0)).max() <= 1e-5 * scale * max(1.0, np.sqrt(len(F)))


@pytest.mark.parametrize("name,n,g", SMALL)
@pytest.mark.parametrize("det", [False, True])
def test_one_step(name, n, g, det):
    w = _w(name, n, g)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp, deterministic=det)
    sim.step(1)
    sim.sync()
    x = sim.positions().cpu().numpy()
    c = sim.field().cpu().numpy()
    X1, c1 = oracle_steps(w, inp, 1)
    assert pos_err(x, X1, w.L, w.periodic) <= 1e-5
    assert field_err(c, c1) <= 1e-5


@pytest.mark.parametrize("name", FULL)
def test_one_step_full_size(name):
    """Full size: positions and field against the oracle's step (1e-5 L,
    1e-5 max|c|); the field also against the oracle's deposit and PDE at the
    device's own new positions, at the same bar."""
    w = W.workload(name)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.step(1)
    sim.sync()
    x = sim.positions().cpu().numpy()
    c = sim.field().cpu().numpy()
    X1, c1 = oracle_steps(w, inp, 1)
    ex, ec = pos_err(x, X1, w.L, w.periodic), field_err(c, c1)
    ecp = field_err(c, field_from_positions(w, inp["c0"], x, inp["species0"]))
    print(f"{name}: position err {ex:.2e} field err {ec:.2e} (at device positions {ecp:.2e})")
    assert ex <= 1e-5
    assert ec <= 1e-5
    assert ecp <= 1e-5


def test_ensemble_256_full_size_sampled_instances():
    """The 256-instance batch at full size (1.41M agents) in the launch
    configuration the benchmark's autotuner picks for it (bins at the contact
    distance, 128-thread work-groups, deposit and PDE of each instance in one
    work-group): neighbour sets at X^0 and one step, then one step from the
    device's state at step 250, checked on the smallest, the largest and two
    other instances, each run alone by the oracle."""
    w = W.workload(W.ENSEMBLE_256)
    inp = W.make_inputs(w)
    cut = max(s.diameter for s in w.species)
    sim = make_sim(w, inp, bin_size=cut * 1.0002, block=128, deposit_mode=3)
    assert sim.info["deposit_path"] == 3 and sim.info["stencil"] == 3
    cnt, hsh = sim.debug_neighbours()
    cnt = cnt.cpu().numpy().astype(np.uint32)
    hsh = hsh.cpu().numpy().view(np.uint64)
    sim.step(1)
    sim.sync()
    x = sim.positions().cpu().numpy()
    c = sim.field().cpu().numpy()
    sizes = np.array([ins.n_agents for ins in w.instances])
    off = np.concatenate([[0], np.cumsum(sizes)])
    G = w.grid_n ** w.dim
    diam = [s.diameter for s in w.species]
    for k in sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 0, 137}):
        a, b = off[k], off[k + 1]
        x0, s0 = inp["x0"][a:b], inp["species0"][a:b]
        oc, oh = oracle.neighbours_f32(w.dim, w.periodic, w.L, x0, s0,
                                       np.arange(b - a, dtype=np.uint32), diam)
        assert np.array_equal(cnt[a:b], oc) and np.array_equal(hsh[a:b], oh), k
        X1, c1, _ = oracle.run(oracle.params(w, k), x0, s0, inp["c0"][k * G:(k + 1) * G], 0, 1)
        assert pos_err(x[a:b], X1, w.L, w.periodic) <= 1e-5, k
        assert field_err(c[k * G:(k + 1) * G], c1) <= 1e-5, k
    # half-way through the benchmark's 500 steps (graph replay), one more
    # step from the device's own state
    sim.use_graph(True)
    sim.step(249)
    sim.sync()
    xs, cs, st = sim.get_state()
    assert st == 250
    xs, cs = xs.cpu().numpy(), cs.cpu().numpy()
    sim.step(1)
    sim.sync()
    x = sim.positions().cpu().numpy()
    c = sim.field().cpu().numpy()
    for k in sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 0, 137}):
        a, b = off[k], off[k + 1]
        X1, c1, _ = oracle.run(oracle.params(w, k), xs[a:b], inp["species0"][a:b],
                               cs[k * G:(k + 1) * G], 250, 1)
        assert pos_err(x[a:b], X1, w.L, w.periodic) <= 1e-5, k
        assert field_err(c[k * G:(k + 1) * G], c1) <= 1e-5, k


@pytest.mark.parametrize("n0", [50, 199])
def test_one_step_3d_blobs_from_clustered_gpu_state(n0):
    """The full 1M-agent 3D run in the benchmark's launch, stepped on the
    device to step n0 (the blobs have collapsed: ~345 neighbours per agent
    at step 75, dense bins on the wave-uniform path).  From the device's
    float32 state at n0: neighbour sets bit-exact, and one more step within
    the per-step bars of the oracle's step from that state with the same
    counter."""
    w = W.workload(W.BLOBS_1M)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.use_graph(True)
    sim.step(n0)
    sim.sync()
    x, c, st = sim.get_state()
    assert st == n0
    x, c = x.cpu().numpy(), c.cpu().numpy()
    cnt, hsh = sim.debug_neighbours()
    sn = dict(inp, x0=x, c0=c)
    ocnt, ohsh = oracle_neighbours(w, sn)
    assert ocnt.mean() > 50
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ocnt)
    assert np.array_equal(hsh.cpu().numpy().view(np.uint64), ohsh)
    sim.step(1)
    sim.sync()
    x1 = sim.positions().cpu().numpy()
    c1 = sim.field().cpu().numpy()
    Xo, co = oracle_steps(w, sn, 1, step0=n0)
    ex, ec = pos_err(x1, Xo, w.L, w.periodic), field_err(c1, co)
    ecp = field_err(c1, field_from_positions(w, c, x1, inp["species0"]))
    print(f"step {n0}: position err {ex:.2e} field err {ec:.2e} (at device positions {ecp:.2e})")
    assert ex <= 1e-5
    assert ec <= 1e-5
    assert ecp <= 1e-5


def test_one_step_later_counter_3d_blobs():
    """Per-step parity at a later step counter and evolved state: the oracle
    evolves the state for 5 steps, both sides take step 5 -> 6 from it."""
    import torch
    w = W.workload(W.BLOBS_1M)
    inp = W.make_inputs(w)
    X5, c5 = oracle_steps(w, inp, 5)
    sim = make_sim(w, inp)
    x32 = torch.from_numpy(X5.astype(np.float32))
    c32 = torch.from_numpy(c5.astype(np.float32))
    sim.set_state(x32, c32, 5)
    sim.step(1)
    sim.sync()
    inp5 = dict(inp, x0=X5.astype(np.float32), c0=c5.astype(np.float32))
    X6, c6 = oracle_steps(w, inp5, 1, step0=5)
    assert pos_err(sim.positions().cpu().numpy(), X6, w.L, True) <= 1e-5
    assert field_err(sim.field().cpu().numpy(), c6) <= 1e-5


@pytest.mark.parametrize("name,steps", [(W.PERIODIC_1K, 100), (W.WALLS_100K, 20),
                                        (W.ADJOINT_50K, 20)])
def test_trajectory(name, steps):
    w = W.workload(name)
    if name != W.PERIODIC_1K:
        w = W.scaled(w, n_agents=20000)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.step(steps)
    sim.sync()
    Xn, cn = oracle_steps(w, inp, steps)
    ex = pos_err(sim.positions().cpu().numpy(), Xn, w.L, w.periodic)
    ec = field_err(sim.field().cpu().numpy(), cn)
    print(f"{name} {steps} steps: position err {ex:.3e} field err {ec:.3e}")
    assert ex <= 1e-5 * steps and ec <= 1e-5 * steps


def _rounded_up_coords(n_cells, inv_h, L):
    """float32 coordinates x just below a node plane k h whose float32
    product x * (1/h) rounds up to the integer k (exactly below it in real
    arithmetic): the cell is k - 1 with offset 1 - tiny."""
    out = []
    for k in range(1, n_cells):
        x = np.float32(k * (L / n_cells))
        for _ in range(4):
            x = np.nextafter(x, np.float32(-1.0), dtype=np.float32)
            if float(x) * float(inv_h) < k and np.float32(x) * np.float32(inv_h) == np.float32(k):
                out.append(x)
    return np.array(out, np.float32)


@pytest.mark.parametrize("dim,periodic,grid_n,det",
                         [(3, True, 48, False), (3, True, 48, True), (2, False, 51, False),
                          (2, True, 37, False)])
def test_deposit_where_quotient_rounds_to_a_node(dim, periodic, grid_n, det):
    """Particle-in-cell deposit (Sect. 2.3) of agents sitting a float32 ulp
    below node planes, where x / h rounds up to the node's index: each
    weight must stay in [0, 1] (no fixed-point wrap of a negative weight).
    The agents do not move (D = 0, chi = 0, k = 0), so the deposit is taken
    at exactly these positions; a source and an uptake species."""
    base = W.workload(W.WALLS_100K)
    sp = (W.Species(0.002, 0.0, 0.0, 1.0, 0.0), W.Species(0.002, 0.0, 0.0, 0.0, 1.0))
    n_cells = grid_n if periodic else grid_n - 1
    L = 1.0
    inv_h = np.float32(n_cells / L)
    xs = _rounded_up_coords(n_cells, inv_h, L)
    assert len(xs) >= 3
    rng = np.random.default_rng(7)
    n = 3 * len(xs) * dim
    x0 = rng.uniform(0.0, L, size=(n, dim)).astype(np.float32)
    for a in range(dim):  # every axis gets every adversarial coordinate
        sl = slice(a * 3 * len(xs), (a + 1) * 3 * len(xs))
        x0[sl, a] = np.tile(xs, 3)
    x0 = np.ascontiguousarray(x0)
    w = W.Workload("rounded_planes", dim, periodic, L, grid_n, 1e-4, 0.0, 1.0, 0.1, 1, sp,
                   (W.Instance(n, 77),), species_rule="halves", c0="sin" if periodic else "cos")
    inp = W.make_inputs(w)
    inp["x0"] = x0
    sim = make_sim(w, inp, deterministic=det)
    sim.step(1)
    sim.sync()
    x = sim.positions().cpu().numpy()
    c = sim.field().cpu().numpy()
    assert np.array_equal(x, x0)
    X1, c1 = oracle_steps(w, inp, 1)
    ec = field_err(c, c1)
    print(f"dim {dim} periodic {periodic} n {grid_n}: {len(xs)} coordinates, field err {ec:.2e}")
    assert ec <= 1e-5
