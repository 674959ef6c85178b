"""Differentiable density-mismatch run: torch.autograd.Function over the
library's forward steps and its reverse sweep (pc_adjoint_segment).

theta = (chi, k, D): chi of every chemotactic species (species whose base
chi is nonzero), the repulsion stiffness and the diffusivity of every
species.  The noise of every step is fixed by the Philox keys, so the loss
is a deterministic function of theta.  The forward keeps a checkpoint of the
state every K steps; the backward replays each segment (recomputing its
states inside the library) from the last to the first.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from .sim import ModelSpec, Sim, SpeciesSpec


def spec_at(base: ModelSpec, theta) -> ModelSpec:
    chi, k, D = (float(v) for v in theta)
    sp = [SpeciesSpec(s.diameter, D, chi if s.chi != 0.0 else 0.0, s.source, s.uptake)
          for s in base.species]
    return dataclasses.replace(base, species=sp, k=k)


class DensityLossRun(torch.autograd.Function):
    """loss(theta) = sum over instances of the smoothed-histogram mismatch of
    the positions after n_steps steps."""

    @staticmethod
    def forward(ctx, theta, base, x0, s0, c0, target, n_steps, K, hist_n, sigma_bins):
        th = theta.detach().cpu().double().numpy()
        if np.any(th == 0.0):
            raise ValueError("theta components must be nonzero (gradients come as scale "
                             "derivatives divided by theta)")
        sim = Sim(spec_at(base, th), x0, s0, c0, adjoint_steps=K)
        ckpts, left = [], int(n_steps)
        while left > 0:
            kk = min(K, left)
            x, c, st = sim.get_state()
            ckpts.append((x, c, st, kk))
            sim.step(kk)
            left -= kk
        loss, dLdX = sim.density_loss(target, hist_n, sigma_bins, grad=True)
        ctx.sim, ctx.ckpts, ctx.dLdX, ctx.theta = sim, ckpts, dLdX, th
        return torch.tensor(float(loss.sum()), dtype=torch.float64)

    @staticmethod
    def backward(ctx, g):
        sim = ctx.sim
        lamX = ctx.dLdX * float(g)
        lamC = torch.zeros(sim.spec.n_nodes, dtype=torch.float32, device=sim.device)
        dth = np.zeros(3)
        for x, c, st, kk in reversed(ctx.ckpts):
            sim.set_state(x, c, st)
            lamX, lamC, d = sim.adjoint_segment(lamX, lamC, kk)
            dth += d.sum(0)
        grad = torch.tensor(dth / ctx.theta, dtype=torch.float64)
        ctx.sim = None
        sim.close()
        return grad, None, None, None, None, None, None, None, None, None


def density_loss_run(theta, base: ModelSpec, x0, s0, c0, target, n_steps: int, K: int = 20,
                     hist_n: int = 64, sigma_bins: float = 2.0) -> torch.Tensor:
    """Differentiable loss(theta); theta is a float64 tensor (chi, k, D)."""
    return DensityLossRun.apply(theta, base, x0, s0, c0, target, n_steps, K, hist_n,
                                sigma_bins)
