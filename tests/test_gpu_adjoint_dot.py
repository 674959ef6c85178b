"""Dot-product (transpose) tests of the reverse-mode kernels, one step.

For the one-step map Phi: (X^n, c^n) -> (X^{n+1}, c^{n+1}) with the noise
fixed by the Philox keys, the library's reverse sweep gives J^T w for a
cotangent w = (w_X, w_c).  With a random direction v = (dX, dc),

    <v, J^T w>  (device, through pc_adjoint_segment over one step)

must equal

    <J v, w>    (FP64 central difference of the oracle's step along v).

The identity part <v, w> is taken off both sides, so the comparison sees
only what the kernels add.  Each case switches on one block of J, so that
one reverse kernel carries the whole difference:

* PDE block c -> c (k_adj_pde): chi = 0, v and w on the field only;
* gradient block c -> X (k_adj_grad and the node-gradient scatter of
  k_adj_agent): v on the field, w on the positions, chi != 0;
* drift and boundary block X -> X (k_adj_agent): k = 0, chi != 0, walls;
* deposit block X -> c (k_adj_agent's deposit adjoint): v on positions,
  w on the field, source and uptake species;
* pair block X -> X (k_adj_pair): chi = 0, k != 0;
* parameter derivatives (chi, k, D scales): <w, dPhi/ds_j> by central
  differences of the oracle's step in s_j.

Positions are perturbed by 1e-9 L (central differences in FP64; at that
step a random direction almost never carries an agent across a cell face
or a contact distance, where the map has kinks).
"""
import dataclasses
import zlib

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_helpers import make_sim

pytestmark = pytest.mark.gpu

EPS_X = 1e-9
EPS_C = 1e-7


def _phi(w, x, sp, c, step0=0):
    """Oracle step of every instance (FP64 state in, FP64 state out)."""
    inp = {"x0": x, "species0": sp, "c0": c}
    X, cc = oracle.run_workload(w, inp, 1, step0=step0)
    return X, cc


def _minimg(d, L, periodic):
    return d - np.rint(d / L) * L if periodic else d


def _jvp(w, x, sp, c, dX, dc, step0=0):
    """(J v) by central differences of the oracle's step."""
    x = x.astype(np.float64)
    c = c.astype(np.float64)
    Xp, cp = _phi(w, x + EPS_X * dX, sp, c + EPS_C * dc, step0)
    Xm, cm = _phi(w, x - EPS_X * dX, sp, c - EPS_C * dc, step0)
    # one scale for both parts: the direction is (EPS_X dX, EPS_C dc) / EPS
    return _minimg(Xp - Xm, w.L, w.periodic), cp - cm


def _case(kind):
    """(workload, v on X?, v on c?, w on X?, w on c?) of one block."""
    if kind == "pde":
        sp = (W.Species(0.01, 1.0, 0.0, 1.0, 0.0), W.Species(0.01, 0.5, 0.0, 0.0, 1.0))
        w = W.Workload("dot_pde", 2, True, 1.0, 40, 1e-4, 100.0, 1.0, 0.3, 1, sp,
                       (W.Instance(2000, 91),), species_rule="halves")
        return w, (0, 1, 0, 1)
    if kind == "pde_walls_3d":
        sp = (W.Species(0.02, 1.0, 0.0, 1.0, 0.0), W.Species(0.02, 0.5, 0.0, 0.0, 2.0))
        w = W.Workload("dot_pde3", 3, False, 1.0, 17, 2e-4, 100.0, 1.0, 0.3, 1, sp,
                       (W.Instance(3000, 92),), species_rule="halves", c0="cos")
        return w, (0, 1, 0, 1)
    if kind == "grad":
        sp = (W.Species(0.01, 1.0, 2.0, 1.0, 0.0),)
        w = W.Workload("dot_grad", 2, True, 1.0, 40, 1e-4, 100.0, 1.0, 0.1, 1, sp,
                       (W.Instance(2000, 93),))
        return w, (0, 1, 1, 0)
    if kind == "grad_walls_3d":
        sp = (W.Species(0.02, 1.0, 2.0, 1.0, 0.0),)
        w = W.Workload("dot_grad3", 3, False, 1.0, 17, 1e-4, 100.0, 1.0, 0.1, 1, sp,
                       (W.Instance(3000, 94),), c0="cos")
        return w, (0, 1, 1, 0)
    if kind == "drift_walls":
        sp = (W.Species(0.01, 1.0, 3.0, 0.0, 0.0),)
        w = W.Workload("dot_drift", 2, False, 1.0, 33, 1e-4, 0.0, 1.0, 0.1, 1, sp,
                       (W.Instance(3000, 95),), c0="cos")
        return w, (1, 0, 1, 0)
    if kind == "deposit":
        sp = (W.Species(0.01, 1.0, 0.0, 1.0, 0.0), W.Species(0.01, 0.5, 0.0, 0.0, 1.0))
        w = W.Workload("dot_dep", 2, True, 1.0, 40, 1e-4, 0.0, 1.0, 0.1, 1, sp,
                       (W.Instance(2000, 96),), species_rule="halves")
        return w, (1, 0, 0, 1)
    if kind == "deposit_walls_3d":
        sp = (W.Species(0.02, 1.0, 0.0, 1.0, 0.0), W.Species(0.02, 0.5, 0.0, 0.0, 1.0))
        w = W.Workload("dot_dep3", 3, False, 1.0, 17, 1e-4, 0.0, 1.0, 0.1, 1, sp,
                       (W.Instance(3000, 97),), species_rule="halves", c0="cos")
        return w, (1, 0, 0, 1)
    if kind == "pair":
        sp = (W.Species(0.03, 1.0, 0.0, 0.0, 0.0), W.Species(0.02, 0.5, 0.0, 0.0, 0.0))
        w = W.Workload("dot_pair", 2, True, 1.0, 32, 1e-4, 300.0, 1.0, 0.1, 1, sp,
                       (W.Instance(3000, 98),), species_rule="halves")
        return w, (1, 0, 1, 0)
    if kind == "pair_3d":
        sp = (W.Species(0.06, 1.0, 0.0, 0.0, 0.0),)
        w = W.Workload("dot_pair3", 3, True, 1.0, 16, 1e-4, 300.0, 1.0, 0.1, 1, sp,
                       (W.Instance(4000, 99),))
        return w, (1, 0, 1, 0)
    raise ValueError(kind)


KINDS = ["pde", "pde_walls_3d", "grad", "grad_walls_3d", "drift_walls", "deposit",
         "deposit_walls_3d", "pair", "pair_3d"]


@pytest.mark.parametrize("kind", KINDS)
def test_one_step_transpose(kind):
    w, (vx, vc, wx, wc) = _case(kind)
    inp = W.make_inputs(w)
    rng = np.random.default_rng(zlib.crc32(kind.encode()))
    N, d, G = w.n_total, w.dim, w.n_nodes
    dX = rng.standard_normal((N, d)) if vx else np.zeros((N, d))
    dc = rng.standard_normal(G) if vc else np.zeros(G)
    wX = rng.standard_normal((N, d)).astype(np.float32) if wx else np.zeros((N, d), np.float32)
    wC = rng.standard_normal(G).astype(np.float32) if wc else np.zeros(G, np.float32)
    sim = make_sim(w, inp, adjoint_steps=1, deterministic=True)
    lx, lc, dth = sim.adjoint_segment(torch.from_numpy(wX), torch.from_numpy(wC), 1)
    lx = lx.cpu().numpy().astype(np.float64)
    lc = lc.cpu().numpy().astype(np.float64)
    wX64, wC64 = wX.astype(np.float64), wC.astype(np.float64)
    # device side: <v, (J^T - I) w>, split by the parts of v
    dev = (EPS_X * (dX * (lx - wX64)).sum() + EPS_C * (dc * (lc - wC64)).sum())
    JX, Jc = _jvp(w, inp["x0"], inp["species0"], inp["c0"], dX, dc)
    # oracle side: <(J - I) v, w> over the same 2 eps scaling (central difference)
    ora = 0.5 * ((wX64 * (JX - 2 * EPS_X * dX)).sum() + (wC64 * (Jc - 2 * EPS_C * dc)).sum())
    # the identity part of each side, for scale
    ident = abs(EPS_X * (dX * wX64).sum() + EPS_C * (dc * wC64).sum())
    print(f"{kind}: <v, (J^T - I) w> device {dev:.9e} oracle {ora:.9e} "
          f"rel {abs(dev - ora) / abs(ora):.2e} (identity part {ident:.3e})")
    assert abs(ora) > 0.0
    assert abs(dev - ora) <= 1e-4 * abs(ora)


@pytest.mark.parametrize("kind", ["grad", "pair", "drift_walls", "pde"])
def test_one_step_parameter_derivatives(kind):
    """<w, dPhi/ds_j> for the scales s of chi, k and D against central
    differences of the oracle's step in theta_j (d/ds_j = theta_j d/dtheta_j)."""
    w, _ = _case(kind)
    w = dataclasses.replace(w, k=w.k if w.k else 50.0)
    inp = W.make_inputs(w)
    rng = np.random.default_rng(5)
    N, d, G = w.n_total, w.dim, w.n_nodes
    wX = rng.standard_normal((N, d)).astype(np.float32)
    wC = rng.standard_normal(G).astype(np.float32)
    sim = make_sim(w, inp, adjoint_steps=1, deterministic=True)
    _, _, dth = sim.adjoint_segment(torch.from_numpy(wX), torch.from_numpy(wC), 1)
    chi = max(s.chi for s in w.species) or 1.0
    theta = np.array([chi, w.k, max(s.D for s in w.species)])

    def f(th):
        wt = oracle.workload_at(w, th)
        # workload_at sets every species' D to theta[2]; keep the per-species
        # ratios by scaling instead
        sc = th / theta
        sp = tuple(dataclasses.replace(s, D=s.D * sc[2], chi=s.chi * sc[0]) for s in w.species)
        wt = dataclasses.replace(wt, species=sp)
        X, c = oracle.run_workload(wt, inp, 1)
        return (wX.astype(np.float64) * X).sum() + (wC.astype(np.float64) * c).sum()

    for j in range(3):
        if theta[j] == 0.0:
            continue
        h = 1e-6 * theta[j]
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        ref = (f(tp) - f(tm)) / (2 * h) * theta[j]
        print(f"{kind} s[{j}]: device {dth[0, j]:.9e} oracle {ref:.9e}")
        if ref == 0.0:
            assert dth[0, j] == 0.0
        else:
            assert abs(dth[0, j] - ref) <= 1e-4 * abs(ref) + 1e-9 * abs(theta[j])
