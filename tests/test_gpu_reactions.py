"""Type switching on the GPU (eq. Chemo_reactions, fixed-step rule of
Sect. 2.1) against the FP64 oracle, through the C ABI.

Bars: with constant rates the switch decision depends only on (step, id,
stream) and the threshold rate * dt, which both sides compare exactly, so
species agree bit for bit over any number of steps.  With a concentration-
dependent rate the GPU forms the threshold in float32, so a decision may
differ only for agents whose uniform lies within 1e-6 of the FP64 threshold.
Positions and field keep the one-step bars of the plain step (1e-5).
"""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import field_err, make_sim, pos_err

pytestmark = pytest.mark.gpu


def _reacting(w, r01=0.0, r01c=0.0, r10=0.0, r10c=0.0):
    s0, s1 = w.species
    sp = (dataclasses.replace(s0, react_to=1, react_rate=r01, react_rate_c=r01c),
          dataclasses.replace(s1, react_to=0, react_rate=r10, react_rate_c=r10c))
    return dataclasses.replace(w, species=sp)


def _w_walls(n=20011, g=129, **rates):
    return _reacting(W.scaled(W.workload(W.WALLS_100K), n_agents=n, grid_n=g), **rates)


def _uniforms(seed, stream, step, n):
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = step
    ctr[:, 1] = np.arange(n, dtype=np.uint32)
    ctr[:, 2] = stream
    ctr[:, 3] = 1
    key = np.tile(np.array([seed & 0xFFFFFFFF, ((seed >> 32) & 0xFFFFFFFF) ^ stream], np.uint32),
                  (n, 1))
    w0 = oracle.philox(ctr, key)[:, 0].astype(np.int64)
    return ((w0 >> 8) | 1).astype(np.float64) / 2.0 ** 24


def _state(sim):
    x, c, _ = sim.get_state()
    return x.cpu().numpy(), c.cpu().numpy()


def test_one_step_with_concentration_dependent_rate():
    w = _w_walls(r01=3e4, r10c=1.5e4)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.step(1)
    sp_gpu = sim.species().cpu().numpy()
    x_gpu, c_gpu = _state(sim)
    Xo, co, spo = oracle.run_workload(w, inp, 1, return_species=True)
    # thresholds in FP64 from the oracle's own interpolation of c^0 at X^0
    p = oracle.params(w)
    X0 = inp["x0"].astype(np.float64)
    cval = oracle.interp(p, inp["c0"].astype(np.float64), X0)
    sp0 = inp["species0"]
    thr = np.where(sp0 == 0, 3e4 * w.dt, 1.5e4 * cval * w.dt)
    u = _uniforms(w.instances[0].seed, 0, 0, w.n_total)
    near = np.abs(u - thr) < 1e-6
    diff = sp_gpu != spo
    assert (spo != sp0).sum() > 200  # switches happened in both directions
    assert ((spo == 1) & (sp0 == 0)).any() and ((spo == 0) & (sp0 == 1)).any()
    assert not diff[sp0 == 0].any()  # constant rate: exact
    assert np.all(near[diff]), np.flatnonzero(diff & ~near)[:10]
    if not diff.any():
        assert pos_err(x_gpu, Xo, w.L, w.periodic) <= 1e-5
        assert field_err(c_gpu, co) <= 1e-5


@pytest.mark.parametrize("graph", [False, True])
def test_constant_rates_species_bit_exact_over_steps(graph):
    w = _w_walls(n=5003, g=65, r01=2e4, r10=1.5e4)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.use_graph(graph)
    steps = 12
    sim.step(steps)
    sp_gpu = sim.species().cpu().numpy()
    x_gpu, c_gpu = _state(sim)
    Xo, co, spo = oracle.run_workload(w, inp, steps, return_species=True)
    assert np.array_equal(sp_gpu, spo)
    assert len(sp_gpu) == w.n_total and 0 < (sp_gpu == 1).sum() < w.n_total
    assert pos_err(x_gpu, Xo, w.L, w.periodic) <= 1e-5 * steps
    assert field_err(c_gpu, co) <= 1e-5 * steps


def test_batched_reactions_equal_instances_run_alone():
    rng = np.random.default_rng(12)
    w = W.scaled(W.workload(W.ENSEMBLE_256), n_agents=list(rng.integers(1, 700, 7)), grid_n=24)
    s = w.species[0]
    sp = (dataclasses.replace(s, react_to=1, react_rate=3e3),
          dataclasses.replace(s, chi=0.0, source=0.0, uptake=0.5, react_to=0, react_rate_c=4e3))
    w = dataclasses.replace(w, species=sp, species_rule="halves")
    inp = W.make_inputs(w)
    sim = make_sim(w, inp, deterministic=True)
    sim.step(6)
    xb, cb = _state(sim)
    sb = sim.species().cpu().numpy()
    off = 0
    G = w.grid_n ** 2
    for k, ins in enumerate(w.instances):
        n = ins.n_agents
        w1 = dataclasses.replace(w, instances=(W.Instance(n, ins.seed, ins.chi_scale, k),))
        one = {"x0": inp["x0"][off:off + n], "species0": inp["species0"][off:off + n],
               "c0": inp["c0"][k * G:(k + 1) * G]}
        alone = make_sim(w1, one, deterministic=True)
        alone.step(6)
        xa, ca = _state(alone)
        assert np.array_equal(alone.species().cpu().numpy(), sb[off:off + n])
        assert np.array_equal(xa, xb[off:off + n])
        assert np.array_equal(ca, cb[k * G:(k + 1) * G])
        off += n
    assert (sb != inp["species0"]).any()


def test_set_species_and_set_state_restore():
    import torch
    w = _w_walls(n=3001, g=33, r01=5e4)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    new = torch.from_numpy((np.arange(w.n_total) % 3 == 0).astype(np.uint8))
    sim.set_species(new)
    assert np.array_equal(sim.species().cpu().numpy(), new.numpy())
    sim.step(4)
    assert not np.array_equal(sim.species().cpu().numpy(), new.numpy())
    sim.set_state(torch.from_numpy(inp["x0"]), torch.from_numpy(inp["c0"]), 0)
    assert np.array_equal(sim.species().cpu().numpy(), new.numpy())
    # the restored run repeats the oracle's run from the new species
    sim.step(3)
    inp2 = dict(inp, species0=new.numpy())
    _, _, spo = oracle.run_workload(w, inp2, 3, return_species=True)
    assert np.array_equal(sim.species().cpu().numpy(), spo)


def test_bad_species_value_reported_and_replaced():
    import torch
    from paper_1805_11007_amd import PcError
    w = _w_walls(n=1000, g=17)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    bad = torch.zeros(w.n_total, dtype=torch.uint8)
    bad[5] = 9
    sim.set_species(bad)
    with pytest.raises(PcError):
        sim.sync()
    assert sim.species().cpu().numpy()[5] == 0
    sim.sync()  # reported once


def test_certain_switch_sets_warning():
    from paper_1805_11007_amd import _lib as LB
    w = _w_walls(n=2000, g=17)
    w = _reacting(w, r01=1.0 / w.dt)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.step(1)
    assert np.all(sim.species().cpu().numpy() == 1)
    assert sim.warnings() & LB.PC_WARN_REACTION


def test_reverse_mode_rejects_switching():
    import torch
    from paper_1805_11007_amd import PcError
    w = _reacting(W.scaled(W.workload(W.ADJOINT_50K), n_agents=2000, grid_n=32), r01=10.0)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp, adjoint_steps=2)
    lx = torch.zeros(w.n_total, 2)
    lc = torch.zeros(w.n_nodes)
    with pytest.raises(PcError):
        sim.adjoint_segment(lx, lc, 1)
