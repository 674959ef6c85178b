"""Ensemble statistics (experiment of Sect. 4, Fig. 1) on the GPU against
the oracle, through the C ABI.

Bars: the per-species histogram counts and totals are integers decided in
float32 on the same float32 positions, so they are bit-exact; the mean
field is within 1e-6 of max|c| of the FP64 mean; along a trajectory the
species are bit-exact (constant switching rate) and the histograms of the
GPU and oracle runs differ only by agents that crossed a bin edge within
the position tolerance.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import field_err, make_sim, pos_err

pytestmark = pytest.mark.gpu


def _check_stats(sim, w, hist_n):
    counts, totals, cm = sim.ensemble_stats(hist_n)
    x = sim.positions().cpu().numpy()
    sp = sim.species().cpu().numpy()
    oc, ot = oracle.species_hist(w.dim, w.L, x, sp, len(w.species), hist_n)
    assert np.array_equal(counts.cpu().numpy().view(np.uint32), oc)
    assert np.array_equal(totals.cpu().numpy().view(np.uint32), ot)
    c = sim.field().cpu().numpy()
    ref = oracle.field_mean(c, w.n_inst)
    assert np.abs(cm.cpu().numpy() - ref).max() <= 1e-6 * max(np.abs(ref).max(), 1e-30)
    return counts.cpu().numpy(), totals.cpu().numpy()


@pytest.mark.parametrize("n_real,hist_n", [(37, 52), (5, 1), (13, 7)])
def test_stats_small_ensembles(n_real, hist_n):
    w = W.fig1_walls_2d(n_real=n_real)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    _check_stats(sim, w, hist_n)
    sim.step(25)
    _check_stats(sim, w, hist_n)


def test_stats_full_fig1_ensemble_conserves_agents():
    w = W.workload(W.FIG1_2000)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.use_graph(True)
    _, tot0 = _check_stats(sim, w, 52)
    assert list(tot0) == [200 * 1000, 200 * 1000]
    sim.step(200)
    counts, tot = _check_stats(sim, w, 52)
    assert tot.sum() == w.n_total and tot[1] > tot0[1]
    per = sim.species().cpu().numpy().reshape(w.n_inst, 200)
    assert per.shape == (2000, 200)  # every realisation keeps its 200 agents


def test_stats_global_atomic_path_3d():
    w = W.scaled(W.workload(W.BLOBS_1M), n_agents=50000, grid_n=32)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    sim.step(3)
    _check_stats(sim, w, 64)   # 64^3 bins: beyond the LDS copy


@pytest.mark.parametrize("n_real", [24, 80])
def test_stats_along_a_trajectory_match_oracle_run(n_real):
    """80 realisations take the per-instance fused deposit + PDE path."""
    w = W.fig1_walls_2d(n_real=n_real)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    assert sim.info["deposit_path"] == (3 if n_real >= 64 else 2)
    steps = 30
    sim.step(steps)
    counts, tot = _check_stats(sim, w, 26)
    Xo, _, spo = oracle.run_workload(w, inp, steps, return_species=True)
    assert np.array_equal(sim.species().cpu().numpy(), spo)
    oc, ot = oracle.species_hist(2, w.L, Xo.astype(np.float32), spo, 2, 26)
    assert np.array_equal(tot.view(np.uint32), ot)
    moved = np.abs(counts.view(np.uint32).astype(np.int64) - oc.astype(np.int64)).sum()
    assert moved <= 2 * max(1, int(0.002 * w.n_total))
    Xo64, co, _ = oracle.run_workload(w, inp, steps, return_species=True)
    x, c, _ = sim.get_state()
    assert pos_err(x.cpu().numpy(), Xo64, w.L, w.periodic) <= 1e-5 * steps
    assert field_err(c.cpu().numpy(), co) <= 1e-5 * steps


def test_fig1_full_size_sampled_realisations_match_oracle():
    """The 2000-realisation batch (per-instance fused deposit + PDE, graph
    replay) against the oracle run of three realisations on their own:
    species bit-exact (constant switching rate), positions within 1e-5 L per
    step, field within 1e-5 max|c| per step."""
    w = W.workload(W.FIG1_2000)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    assert sim.info["deposit_path"] == 3
    sim.use_graph(True)
    steps = 12
    sim.step(steps)
    x, c, _ = sim.get_state()
    x, c = x.cpu().numpy(), c.cpu().numpy()
    sp = sim.species().cpu().numpy()
    G = w.grid_n ** 2
    for k in (0, 777, 1999):
        a, n = 200 * k, 200
        p = oracle.params(w, k)
        Xo, co, _, so = oracle.run(p, inp["x0"][a:a + n], inp["species0"][a:a + n],
                                   inp["c0"][k * G:(k + 1) * G], 0, steps, return_species=True)
        assert np.array_equal(sp[a:a + n], so), k
        assert pos_err(x[a:a + n], Xo, w.L, w.periodic) <= 1e-5 * steps, k
        assert field_err(c[k * G:(k + 1) * G], co) <= 1e-5 * steps, k
