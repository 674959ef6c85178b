"""The autotuner: every candidate it can pick gives the same neighbour sets
and one-step result (within the parity bars), and its cache round-trips."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_helpers import field_err, oracle_steps, pos_err

pytestmark = pytest.mark.gpu


def test_autotune_picks_a_valid_configuration(tmp_path, monkeypatch):
    from paper_1805_11007_amd import ModelSpec, Sim
    from paper_1805_11007_amd import autotune as AT
    monkeypatch.setenv("PC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    w = W.scaled(W.workload(W.ENSEMBLE_256), n_agents=[900, 40, 3000, 1, 250], grid_n=48)
    inp = W.make_inputs(w)
    x0, s0, c0 = (torch.from_numpy(inp[k]) for k in ("x0", "species0", "c0"))
    spec, rep = AT.tune(ModelSpec.from_workload(w), x0, s0, c0, steps=4)
    assert "best" in rep and spec.block in AT.CANDIDATE_BLOCKS
    assert len([t for t in rep["trials"] if "ms_per_step" in t]) >= 6
    spec2, rep2 = AT.tune(ModelSpec.from_workload(w), x0, s0, c0, steps=4)
    assert "cached" in rep2 and spec2.bin_size == spec.bin_size and spec2.block == spec.block
    sim = Sim(spec, x0, s0, c0)
    sim.step(1)
    X1, c1 = oracle_steps(w, inp, 1)
    assert pos_err(sim.positions().cpu().numpy(), X1, 1.0, True) <= 1e-5
    assert field_err(sim.field().cpu().numpy(), c1) <= 1e-5


@pytest.mark.parametrize("bin_mult,block", [(1.0, 64), (1.25, 512), (2.0, 128), (3.0, 1024)])
def test_every_candidate_is_parity_green(bin_mult, block):
    from paper_1805_11007_amd import ModelSpec, Sim
    w = W.scaled(W.workload(W.BLOBS_1M), n_agents=30000, grid_n=32)
    inp = W.make_inputs(w)
    spec = ModelSpec.from_workload(w, bin_size=bin_mult * 0.004 * (1 + 2e-4), block=block)
    sim = Sim(spec, torch.from_numpy(inp["x0"]), torch.from_numpy(inp["species0"]),
              torch.from_numpy(inp["c0"]))
    assert sim.info["stencil"] == (2 if bin_mult >= 2 else 3)
    import oracle
    from gpu_helpers import oracle_neighbours
    cnt, hsh = sim.debug_neighbours()
    ocnt, ohsh = oracle_neighbours(w, inp)
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ocnt)
    assert np.array_equal(hsh.cpu().numpy().view(np.uint64), ohsh)
    sim.step(1)
    X1, c1 = oracle_steps(w, inp, 1)
    assert pos_err(sim.positions().cpu().numpy(), X1, 1.0, True) <= 1e-5
    assert field_err(sim.field().cpu().numpy(), c1) <= 1e-5


def test_autotune_times_states_along_the_run(tmp_path, monkeypatch):
    """With a horizon the candidates are timed from the states at the start,
    middle and end of the run, cached under their own key, and the choice
    still reproduces the oracle's step."""
    from paper_1805_11007_amd import ModelSpec, Sim
    from paper_1805_11007_amd import autotune as AT
    monkeypatch.setenv("PC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    w = W.scaled(W.workload(W.BLOBS_1M), n_agents=20000, grid_n=24)
    inp = W.make_inputs(w)
    x0, s0, c0 = (torch.from_numpy(inp[k]) for k in ("x0", "species0", "c0"))
    spec, rep = AT.tune(ModelSpec.from_workload(w), x0, s0, c0, steps=3, horizon=30,
                        bins=(1.0, 2.0), blocks=(64, 128))
    assert rep["states_at_steps"] == [0, 15, 27]
    assert any(t.get("deposit_mode") == 4 for t in rep["trials"])   # the slab path is tried
    _, rep0 = AT.tune(ModelSpec.from_workload(w), x0, s0, c0, steps=3, bins=(1.0,),
                      blocks=(128,))
    assert "best" in rep0                     # a horizon-0 tuning is a separate entry
    _, rep2 = AT.tune(ModelSpec.from_workload(w), x0, s0, c0, steps=3, horizon=30)
    assert rep2["cached"]["block"] == spec.block
    sim = Sim(spec, x0, s0, c0)
    sim.step(1)
    X1, c1 = oracle_steps(w, inp, 1)
    assert pos_err(sim.positions().cpu().numpy(), X1, 1.0, True) <= 1e-5
    assert field_err(sim.field().cpu().numpy(), c1) <= 1e-5
