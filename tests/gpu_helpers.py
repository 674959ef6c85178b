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


def deposit_rounding_tol(w, x32, species, c_max):
    """Per-node bound (flat, instance-major like the field) of the difference
    that float32 rounding of the particle-in-cell weights can make in one
    step's field.  The device forms t = x / h - i0 with one rounding
    (fma(x, 1/h, -i0), 1/h exact on these grids), so t is off by at most
    2^-24, each factor 1 - t or t by 2 ulps, and the product of an agent's
    d factors by about 2 d 2^-24.  Node l takes
    dt q_a W / (h^d v_l) from every agent a whose cell has l as a corner,
    with q_a = source + uptake * max|c| (the uptake acts through upsilon c).
    The largest bound of a node's 3^d neighbourhood is taken, since PDE
    substeps spread a node's difference to its neighbours."""
    n, d = w.grid_n, w.dim
    h = w.L / n if w.periodic else w.L / (n - 1)
    inv_h = np.float32(1.0 / h)
    top = np.float32(n - 1 if w.periodic else n - 2)
    src = np.array([s.source for s in w.species])
    upt = np.array([s.uptake for s in w.species])
    G = n ** d
    out = np.empty(w.n_inst * G)
    off = 0
    for k, ins in enumerate(w.instances):
        x = np.asarray(x32[off:off + ins.n_agents], np.float32)
        sp = np.asarray(species[off:off + ins.n_agents])
        off += ins.n_agents
        s = np.maximum(x * inv_h, np.float32(0.0))
        i0 = np.minimum(np.floor(s), top).astype(np.int64)
        cell = i0[:, 0] + n * i0[:, 1] + (n * n * i0[:, 2] if d == 3 else 0)
        q = src[sp] + upt[sp] * c_max
        acc = np.bincount(cell, weights=q, minlength=G).reshape((n,) * d)  # [z][y][x]
        for ax in range(d):  # node l gathers cells l - 1 and l along each axis
            sh = np.roll(acc, 1, axis=ax)
            if not w.periodic:
                idx = [slice(None)] * d
                idx[ax] = 0
                sh[tuple(idx)] = 0.0
            acc = acc + sh
        inv_v = np.ones((n,) * d)
        if not w.periodic:
            for ax in range(d):
                for e in (0, n - 1):
                    idx = [slice(None)] * d
                    idx[ax] = e
                    inv_v[tuple(idx)] *= 2.0
        b = w.dt * inv_v / h ** d * acc * 2.0 * d * 2.0 ** -24
        for ax in range(d):
            pad = [(0, 0)] * d
            pad[ax] = (1, 1)
            bp = np.pad(b, pad, mode="wrap" if w.periodic else "edge")
            sl = lambda a, lo: tuple(slice(lo, lo + n) if i == ax else slice(None) for i in range(d))
            b = np.maximum(np.maximum(bp[sl(None, 0)], bp[sl(None, 1)]), bp[sl(None, 2)])
        out[k * G:(k + 1) * G] = b.reshape(-1)
    return out


def field_ok(c_gpu, c_ref, w, x32, species):
    """Field bar of a whole step: 1e-5 max|c| plus the deposit-weight
    rounding bound of each node."""
    c_ref = np.asarray(c_ref, np.float64)
    cmax = np.abs(c_ref).max()
    tol = 1e-5 * cmax + deposit_rounding_tol(w, x32, species, cmax)
    diff = np.abs(np.asarray(c_gpu, np.float64) - c_ref)
    worst = int(np.argmax(diff / tol))
    print(f"field: max |diff| {diff.max():.3e} (max|c| {cmax:.3e}); at the node nearest "
          f"its bound diff {diff[worst]:.3e} vs bound {tol[worst]:.3e}")
    return bool(np.all(diff <= tol))


def field_from_positions(w, c0, X, species):
    """The oracle's particle-in-cell deposit at positions X (promoted to FP64)
    and its PDE step from c0, instance by instance: the field a step gives
    from those positions.  Comparing the device's field with this one at the
    device's own new positions separates the field's arithmetic from the
    positions' (checked on their own)."""
    G = w.grid_n ** w.dim
    out, off = [], 0
    for k, ins in enumerate(w.instances):
        n = ins.n_agents
        p = oracle.params(w, k)
        Ss, Su = oracle.deposit(p, np.asarray(X[off:off + n], np.float64), species[off:off + n])
        out.append(oracle.pde(p, c0[k * G:(k + 1) * G], Ss, Su))
        off += n
    return np.concatenate(out)
