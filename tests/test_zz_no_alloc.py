"""The allocation-free loss entry point (pc_density_loss_noalloc) against
pc_density_loss, through the C ABI: two calls in a row on one GPU, the
second with fewer agents and a smaller histogram, so that the static
scratch left by the first call must not leak into the second."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_helpers import make_sim

pytestmark = pytest.mark.gpu


def _case(n, g, hist_n, steps):
    w = W.scaled(W.workload(W.ADJOINT_50K), n_agents=n, grid_n=g)
    inp = W.make_inputs(w)
    tw = W.scaled(W.adjoint_2d(chi=1.5, k=800, D=0.8, seed=2005), n_agents=n, grid_n=g)
    target = oracle.target_hist(tw, W.make_inputs(tw), steps, hist_n, 2.0)
    sim = make_sim(w, inp)
    sim.step(steps)
    return w, sim, torch.from_numpy(target.astype(np.float32)).cuda()


@pytest.mark.parametrize("first,second", [((8000, 64, 64, 3), (2000, 32, 24, 2))])
def test_noalloc_loss_matches_the_work_buffer_entry_point(first, second):
    for n, g, hist_n, steps in (first, second):
        w, sim, target = _case(n, g, hist_n, steps)
        loss_ref, g_ref = sim.density_loss(target, hist_n, 2.0, grad=True)
        dLdX = torch.empty(w.n_total, 2, dtype=torch.float32, device="cuda")
        before = torch.cuda.memory_allocated()
        loss = sim.density_loss_noalloc(target, hist_n, 2.0, dLdX)
        assert torch.cuda.memory_allocated() == before
        # same kernels on the same inputs: the gradient bit for bit; the loss
        # is an FP64 sum whose work-group partials meet in device atomics, so
        # its last bits follow their order
        assert np.all(np.abs(loss - loss_ref) <= 1e-12 * np.abs(loss_ref))
        assert torch.equal(dLdX, g_ref)
        # and the loss against the oracle's
        X = sim.positions().cpu().numpy().astype(np.float64)
        lo = oracle.density_loss(2, 1.0, X, target.cpu().numpy().astype(np.float64), hist_n, 2.0)
        assert abs(loss[0] - lo) <= 1e-4 * lo
        sim.close()


def test_noalloc_loss_rejects_what_exceeds_its_scratch():
    from paper_1805_11007_amd import PcError
    w = W.scaled(W.workload(W.BLOBS_1M), n_agents=3000, grid_n=16)
    inp = W.make_inputs(w)
    sim = make_sim(w, inp)
    target = torch.zeros(64 ** 3, dtype=torch.float32, device="cuda")
    with pytest.raises(PcError) as e:
        sim.density_loss_noalloc(target, 64, 2.0)
    assert e.value.code == -3   # PC_ENOSPACE
    # a histogram that fits still works on the same handle
    t2 = torch.zeros(16 ** 3, dtype=torch.float32, device="cuda")
    loss = sim.density_loss_noalloc(t2, 16, 1.0)
    ref, _ = sim.density_loss(t2, 16, 1.0, grad=False)
    assert np.all(np.abs(loss - ref) <= 1e-12 * np.abs(ref))
    sim.close()
