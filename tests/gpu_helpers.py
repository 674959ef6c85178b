"""Shared helpers of the GPU parity tests (GPU library vs FP64 oracle)."""
from __future__ import annotations

import numpy as np

import oracle
import workloads as W


def make_sim(w, inp, adjoint_steps=0, **over):
    import torch
    from paper_1805_11007_amd import ModelSpec, Sim
    spec = ModelSpec.from_workload(w, **over)
    return Sim(spec, torch.from_numpy(inp["x0"]), torch.from_numpy(inp["species0"]),
               torch.from_numpy(inp["c0"]), device="cuda:0", adjoint_steps=adjoint_steps)


def pos_err(x_gpu, x_ref, L, periodic):
    d = np.asarray(x_gpu, np.float64) - np.asarray(x_ref, np.float64)
    if periodic:
        d -= np.rint(d / L) * L
    return np.abs(d).max() / L


def field_err(c_gpu, c_ref):
    c_ref = np.asarray(c_ref, np.float64)
    return np.abs(np.asarray(c_gpu, np.float64) - c_ref).max() / max(np.abs(c_ref).max(), 1e-300)


def oracle_neighbours(w, inp):
    """float32 neighbour counts / hashes of every instance (id order)."""
    cnts, hs = [], []
    off = 0
    diam = [s.diameter for s in w.species]
    for ins in w.instances:
        n = ins.n_agents
        c, h = oracle.neighbours_f32(w.dim, w.periodic, w.L, inp["x0"][off:off + n],
                                     inp["species0"][off:off + n], np.arange(n, dtype=np.uint32),
                                     diam)
        cnts.append(c)
        hs.append(h)
        off += n
    return np.concatenate(cnts), np.concatenate(hs)


def oracle_forces(w, inp):
    Fs, off = [], 0
    for k, ins in enumerate(w.instances):
        n = ins.n_agents
        Fs.append(oracle.forces(oracle.params(w, k), inp["x0"][off:off + n].astype(np.float64),
                                inp["species0"][off:off + n]))
        off += n
    return np.concatenate(Fs)


def oracle_steps(w, inp, n_steps, step0=0):
    return oracle.run_workload(w, inp, n_steps, step0=step0)
