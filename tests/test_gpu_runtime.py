"""GPU tests of the library's runtime behaviour: determinism, batching,
graph replay, checkpoint / resume, error paths and edge cases."""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import field_err, make_sim, oracle_neighbours, oracle_steps, pos_err

pytestmark = pytest.mark.gpu


def _state(sim):
    return sim.positions().cpu().numpy(), sim.field().cpu().numpy()


def test_deterministic_mode_bitwise_repeatable():
    w = W.scaled(W.workload(W.BLOBS_1M), n_agents=60000, grid_n=40)
    inp = W.make_inputs(w)
    a = make_sim(w, inp, deterministic=True)
    b = make_sim(w, inp, deterministic=True)
    a.step(7)
    b.step(7)
    xa, ca = _state(a)
    xb, cb = _state(b)
    assert np.array_equal(xa, xb) and np.array_equal(ca, cb)


def test_batch_equals_instances_run_alone():
    """Each instance of a batch evolves exactly as it does alone (same seed
    and noise stream), bit for bit in deterministic mode; the batch also
    matches the oracle."""
    rng = np.random.default_rng(11)
    w = W.scaled(W.workload(W.ENSEMBLE_256), n_agents=list(rng.integers(1, 700, 9)), grid_n=24)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp, deterministic=True)
    sim.step(5)
    xb, cb = _state(sim)
    off = 0
    G = w.grid_n ** 2
    for k, ins in enumerate(w.instances):
        n = ins.n_agents
        w1 = W.Workload(**{**w.__dict__, "instances": (W.Instance(n, ins.seed, ins.chi_scale, k),)})
        one = {"x0": inp["x0"][off:off + n], "species0": inp["species0"][off:off + n],
               "c0": inp["c0"][k * G:(k + 1) * G]}
        alone = make_sim(w1, one, deterministic=True)
        alone.step(5)
        xa, ca = _state(alone)
        assert np.array_equal(xa, xb[off:off + n])
        assert np.array_equal(ca, cb[k * G:(k + 1) * G])
        off += n
    Xo, co = oracle_steps(w, inp, 5)
    assert pos_err(xb, Xo, 1.0, True) <= 5e-5
    assert field_err(cb, co) <= 5e-5


def test_graph_replay_equals_eager():
    w = W.scaled(W.workload(W.PERIODIC_1K), n_agents=2000)
    inp = W.make_inputs(w)
    a = make_sim(w, inp, deterministic=True)
    b = make_sim(w, inp, deterministic=True)
    b.use_graph(True)
    a.step(9)
    b.step(9)
    a.sync(); b.sync()
    xa, ca = _state(a)
    xb, cb = _state(b)
    assert np.array_equal(xa, xb) and np.array_equal(ca, cb)
    # several replays with eager work and syncs in between stay equal
    for _ in range(3):
        a.step(4)
        b.step(4)
        _ = a.positions().sum().item()
        _ = b.positions().sum().item()
    assert np.array_equal(_state(a)[0], _state(b)[0])
    assert np.array_equal(_state(a)[1], _state(b)[1])


def test_checkpoint_resume_bitwise():
    w = W.scaled(W.workload(W.ADJOINT_50K), n_agents=5000, grid_n=64)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp, deterministic=True)
    sim.step(3)
    x, c, st = sim.get_state()
    assert st == 3
    sim.step(4)
    x1, c1 = _state(sim)
    sim.set_state(x, c, st)
    sim.step(4)
    x2, c2 = _state(sim)
    assert np.array_equal(x1, x2) and np.array_equal(c1, c2)


def test_species_and_warnings():
    w = W.scaled(W.workload(W.WALLS_100K), n_agents=5000, grid_n=65)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    assert np.array_equal(sim.species().cpu().numpy(), inp["species0"])
    from paper_1805_11007_amd._lib import PC_WARN_DT_RULE
    assert sim.warnings() & PC_WARN_DT_RULE  # sqrt(2*2*1e-6) = 0.002 = d for species 0


def test_nonfinite_field_raises_enonfinite_at_sync():
    """A NaN in c0 reaches the PDE (and the drift of agents near it); the
    kernels latch the non-finite flag and pc_sync reports PC_ENONFINITE
    once, then clears it."""
    import torch
    from paper_1805_11007_amd import PcError
    from paper_1805_11007_amd._lib import PC_ENONFINITE
    w = W.scaled(W.workload(W.PERIODIC_1K), n_agents=2000, grid_n=32)
    inp = W.make_inputs(w)
    c0 = inp["c0"].copy()
    c0[5 * 32 + 7] = np.nan
    sim = make_sim(w, dict(inp, c0=c0))
    sim.sync()                       # creation itself reads no field value
    sim.step(1)
    with pytest.raises(PcError) as e:
        sim.sync()
    assert e.value.code == PC_ENONFINITE
    sim.sync()                       # reported once, then cleared
    # a finite state restored: further steps are clean
    sim.set_state(torch.from_numpy(inp["x0"]), torch.from_numpy(inp["c0"]), 0)
    sim.step(2)
    sim.sync()


def test_positivity_warning():
    """dt' (gamma + upsilon) >= 1 at a node sets PC_WARN_POSITIVITY."""
    import dataclasses
    from paper_1805_11007_amd._lib import PC_WARN_POSITIVITY
    w = W.scaled(W.workload(W.PERIODIC_1K), n_agents=500, grid_n=16)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.step(2)
    assert not sim.warnings() & PC_WARN_POSITIVITY
    w2 = dataclasses.replace(w, gamma=2.0 / w.dt)   # dt gamma = 2
    sim2 = make_sim(w2, inp)
    sim2.step(1)
    assert sim2.warnings() & PC_WARN_POSITIVITY


def test_walls_keep_agents_in_box():
    w = W.scaled(W.workload(W.WALLS_100K), n_agents=20000, grid_n=65)
    inp = W.make_inputs(w)
    x0 = inp["x0"].copy()
    x0[:500] = 0.0
    x0[500:1000] = 1.0
    inp = dict(inp, x0=x0)
    sim = make_sim(w, inp)
    for _ in range(5):
        sim.step(4)
        x = sim.positions().cpu().numpy()
        assert x.min() >= 0.0 and x.max() <= 1.0
    sim.sync()


def test_edge_cases_single_agent_and_one_bin_pileup():
    # one agent
    w = W.scaled(W.workload(W.PERIODIC_1K), n_agents=1)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.step(3)
    X, c = oracle_steps(w, inp, 3)
    assert pos_err(sim.positions().cpu().numpy(), X, 1.0, True) <= 3e-5
    # 300 agents piled up inside one bin, plus agents on bin faces and at 0 / L^-
    w = W.scaled(W.workload(W.PERIODIC_1K), n_agents=400)
    inp = W.make_inputs(w)
    x0 = inp["x0"].copy()
    x0[:300] = np.float32(0.5) + np.random.default_rng(1).uniform(0, 0.004, (300, 2)).astype(np.float32)
    x0[300:310] = 0.0
    x0[310:320] = np.nextafter(np.float32(1.0), np.float32(0.0))
    x0[320:330, 0] = np.float32(0.25)
    inp = dict(inp, x0=x0)
    sim = make_sim(w, inp)
    cnt, hsh = sim.debug_neighbours()
    ocnt, ohsh = oracle_neighbours(w, inp)
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ocnt)
    assert np.array_equal(hsh.cpu().numpy().view(np.uint64), ohsh)
    sim.step(1)
    X, c = oracle_steps(w, inp, 1)
    assert pos_err(sim.positions().cpu().numpy(), X, 1.0, True) <= 1e-5
    assert field_err(sim.field().cpu().numpy(), c) <= 1e-5


def test_cell_list_with_more_than_8192_scan_tiles():
    """265^3 bins + 1 = 9087 scan tiles of 2048 bins: the tile-sum scan runs
    in two passes of 8192 with a ragged tail.  Neighbour sets stay bit-exact
    against the float32 brute force, at creation and after the cell list has
    been rebuilt by the steps (checked on the GPU's own positions)."""
    w = W.scaled(W.workload(W.BLOBS_1M), n_agents=150000, grid_n=32)
    w = dataclasses.replace(w, species=(dataclasses.replace(w.species[0], diameter=0.0037),))
    inp = W.make_inputs(w)
    sim = make_sim(w, inp, bin_size=1.0 / 265.5)
    assert sim.info["n_bins_total"] == 265 ** 3
    assert -(-(265 ** 3 + 1) // 2048) == 9087
    cnt, hsh = sim.debug_neighbours()
    ocnt, ohsh = oracle_neighbours(w, inp)
    assert ocnt.sum() > 100000
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ocnt)
    assert np.array_equal(hsh.cpu().numpy().view(np.uint64), ohsh)
    sim.step(3)
    x = sim.positions().cpu().numpy()
    cnt, hsh = sim.debug_neighbours()
    ocnt, ohsh = oracle_neighbours(w, dict(inp, x0=x))
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ocnt)
    assert np.array_equal(hsh.cpu().numpy().view(np.uint64), ohsh)


def test_wave_across_bin_rows_with_more_than_1024_bins_per_side():
    """1100 bins per side; 32 agents in bin (1030, 5) and 32 in bin (6, 6)
    form one wave in cell order.  A bin id packed as x + 1024 y is the same
    for both bins, so a wave-uniform test built on it would give the second
    half the first half's stencil and lose its neighbours."""
    w = W.scaled(W.workload(W.PERIODIC_1K), n_agents=64)
    w = dataclasses.replace(w, species=(dataclasses.replace(w.species[0], diameter=0.0009),))
    inp = W.make_inputs(w)
    rng = np.random.default_rng(7)
    x0 = np.empty((64, 2), np.float32)
    x0[:32] = ((np.array([1030.0, 5.0]) + rng.uniform(0.05, 0.95, (32, 2))) / 1100).astype(np.float32)
    x0[32:] = ((np.array([6.0, 6.0]) + rng.uniform(0.05, 0.95, (32, 2))) / 1100).astype(np.float32)
    assert 1030 + 1024 * 5 == 6 + 1024 * 6
    inp = dict(inp, x0=x0)
    sim = make_sim(w, inp, bin_size=1.0 / 1100.5)
    assert sim.info["bins_per_axis"] == 1100
    cnt, hsh = sim.debug_neighbours()
    ocnt, ohsh = oracle_neighbours(w, inp)
    assert ocnt[:32].sum() > 32 and ocnt[32:].sum() > 32
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ocnt)
    assert np.array_equal(hsh.cpu().numpy().view(np.uint64), ohsh)
    sim.step(1)
    X, c = oracle_steps(w, inp, 1)
    assert pos_err(sim.positions().cpu().numpy(), X, 1.0, True) <= 1e-5


def test_error_paths():
    import torch
    from paper_1805_11007_amd import ModelSpec, PcError, Sim
    w = W.scaled(W.workload(W.PERIODIC_1K), n_agents=100)
    inp = W.make_inputs(w)
    bad = inp["species0"].copy()
    bad[5] = 3
    with pytest.raises(PcError):
        Sim(ModelSpec.from_workload(w), torch.from_numpy(inp["x0"]), torch.from_numpy(bad),
            torch.from_numpy(inp["c0"]))
    with pytest.raises(PcError):
        Sim(ModelSpec.from_workload(w, pde_substeps=1, dt=1e-2), torch.from_numpy(inp["x0"]),
            torch.from_numpy(inp["species0"]), torch.from_numpy(inp["c0"]))


def _dep_case(name, n, g):
    import dataclasses
    if name == "3d_walls":
        return dataclasses.replace(W.scaled(W.workload(W.BLOBS_1M), n_agents=n, grid_n=g),
                                   periodic=False, c0="cos")
    if name == "3d_substeps":
        # three PDE substeps: the slab path stores its sums (no fused PDE)
        return dataclasses.replace(W.scaled(W.workload(W.BLOBS_1M), n_agents=n, grid_n=g),
                                   pde_substeps=3)
    if name == "3d_batch":
        w = W.scaled(W.workload(W.BLOBS_1M), n_agents=[n, n // 3, 7], grid_n=g)
        return dataclasses.replace(w, species=(W.Species(0.004, 1.0, 1.0, 1.0, 0.0),
                                               W.Species(0.006, 0.5, 2.0, 0.3, 1.0)),
                                   species_rule="halves")
    if name == "3d_uniform_sparse":
        # agents far sparser than bins: a 1024-agent work-group touches more
        # node rows than the row-window table holds (the overflow path)
        import dataclasses
        return dataclasses.replace(W.scaled(W.workload(W.BLOBS_1M), n_agents=n, grid_n=g),
                                   layout="uniform")
    if name == W.ENSEMBLE_256:
        return W.scaled(W.workload(W.ENSEMBLE_256),
                        n_agents=list(np.random.default_rng(7).integers(1, 600, 70)), grid_n=g)
    if name == W.FIG1_2000:
        return W.fig1_walls_2d(n_real=n)
    return W.scaled(W.workload(name), n_agents=n, grid_n=g)


@pytest.mark.parametrize("name,n,g,modes", [
    (W.BLOBS_1M, 40000, 32, (2, 4)), (W.WALLS_100K, 20011, 129, (2, 4)),
    (W.BLOBS_1M, 400000, 200, (2, 4)), ("3d_substeps", 30011, 40, (2, 4)),
    ("3d_uniform_sparse", 60000, 64, (2, 4)), ("3d_walls", 30011, 33, (2, 4)),
    ("3d_batch", 9001, 20, (2, 4)),
    (W.PERIODIC_1K, 3001, 37, (2, 3, 4)), (W.ENSEMBLE_256, None, 24, (2, 3, 4)),
    (W.ADJOINT_50K, 3000, 32, (2, 3, 4)), (W.FIG1_2000, 70, None, (2, 3, 4))])
def test_deposit_modes_bitwise_equal(name, n, g, modes):
    """The deposit is an integer sum: LDS-aggregated, direct-atomic,
    per-instance fused (deposit + PDE substeps in one work-group) and
    owner-computes slab (gathered through the cell list of X^{n+1}, fused
    with a single PDE substep) paths give the same bits, step after step.
    The slab path runs with its default hand-over threshold, with every
    slab of more than one agent handed to the agent-parallel pass, and with
    a threshold that splits the slabs into both kinds.  On the 200^3 grid
    (5,000 slabs) the handed-over chunks outnumber the hand-over kernel's
    resident work-groups, which then take several chunks each."""
    w = _dep_case(name, n, g)
    inp = W.make_inputs(w)
    a = make_sim(w, inp, deterministic=True, deposit_mode=1)
    assert a.info["deposit_path"] == 1
    a.step(7)
    xa, ca = _state(a)
    runs = [(m, 0) for m in modes] + [(4, 1), (4, 150)] * (4 in modes)
    for m, split in runs:
        b = make_sim(w, inp, deterministic=True, deposit_mode=m, slab_split=split)
        assert b.info["deposit_path"] == (5 if m == 4 else m)
        b.step(7)
        xb, cb = _state(b)
        assert np.array_equal(xa, xb) and np.array_equal(ca, cb), (m, split)
        b.close()


def test_slab_path_default_in_3d_and_rejected_for_bins_far_finer_than_the_grid():
    from paper_1805_11007_amd import PcError
    w = W.scaled(W.workload(W.BLOBS_1M), n_agents=2000, grid_n=24)
    assert make_sim(w, W.make_inputs(w)).info["deposit_path"] == 5
    # 6^3 grid with bins of side 0.004 (249 per axis): ~42 bins per cell,
    # more bin layers per slab than its run table holds
    w = W.scaled(W.workload(W.BLOBS_1M), n_agents=2000, grid_n=6)
    side = 0.004 * 1.0002
    sim = make_sim(w, W.make_inputs(w), bin_size=side)
    assert sim.info["bins_per_axis"] == 249 and sim.info["deposit_path"] != 5
    with pytest.raises(PcError):
        make_sim(w, W.make_inputs(w), bin_size=side, deposit_mode=4)


def test_fused_path_chosen_for_many_small_instances_and_rejected_when_too_big():
    from paper_1805_11007_amd import PcError
    w = W.fig1_walls_2d(n_real=64)
    assert make_sim(w, W.make_inputs(w)).info["deposit_path"] == 3
    w = W.scaled(W.workload(W.BLOBS_1M), n_agents=1000, grid_n=64)  # 64^3 sums do not fit in LDS
    with pytest.raises(PcError):
        make_sim(w, W.make_inputs(w), deposit_mode=3)
