#!/usr/bin/env python3
"""Benchmark of the hybrid chemotaxis step on one MI355X.

Workload: the 3D periodic run with 1,000,000 agents in 8 Gaussian blobs on a
128^3 chemical grid (dt = 1e-7), stepped from its initial state with the
bin side and work-group size the autotuner picks for that run.  W warm-up
steps run first on the same handle, the state is then restored to the
initial condition and exactly K steps are timed (HIP-graph replay, inputs
already resident in HBM).  One JSON line is printed with:

* value: particle-steps/s of the whole timed region;
* roofline: the dominant kernel of the timed steps against the 8 TB/s HBM
  peak: its algorithmic bytes per launch over its mean launch time (HIP
  events between the stages of each step, on the library's stream, over
  the same K steps from the same state), with its rocprofv3 counter bytes;
* step_hbm: the whole step against HBM: the algorithmic floor of a step
  (positions in and out, ids, the field and its deposits) over the step
  time, and the counter bytes of all the step's kernels over the same time;
* cpu_baseline: the FP64 oracle timed on the host cores on a bounded sample
  of the same workload (all threads, and one thread).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = ("particle-steps/s (3D, 1M cells) + % HBM roofline; fwd+bwd and ensemble vs plain")
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3      # MI355X FP32 vector, counting packed (dual-issue) FMA
FP32_ATTAINABLE_TFLOPS = 78.6  # without packed FP32 instructions (this build disables them)

# Algorithmic float operations of the particle update, by definition of what
# it computes: per neighbour pair, the float32 distance (3 sub, 3 mul, 2 add),
# the test, and the force k (d - r)/r applied to dx (rsqrt, 4 fused
# multiply-adds = 8) -> 18; per agent, the interpolated centred-difference
# gradient (24 differences, 8 trilinear weights, 24 multiply-adds ~ 90), the
# Box-Muller normals (~15), the update and boundary (~25), the next bin
# (~10) -> 140.  Integer Philox work is not counted.
FLOP_PER_PAIR, FLOP_PER_AGENT = 18.0, 140.0

# rocprofv3 FETCH_SIZE and WRITE_SIZE of the kernels of one step on the 1M-
# agent 3D workload, over the window the default run times (the first 20
# steps after 5 warm-up steps; each counter in its own run, FETCH_SIZE scaled
# by 2.0 and WRITE_SIZE by 1.0 from a plain device copy).  Bytes per step
# (summed over the step's kernels) and per launch of the update kernel,
# with the tuned choice of that run (bin side = cutoff, 64-thread agent
# work-groups, slab deposit).  Valid only for the kernel sources they were
# taken with (a hash of every file under csrc/), for that workload and that
# deposit path; reported as null otherwise.
COUNTER_STEP_BYTES = 325134723.6
COUNTER_UPDATE_BYTES = 78311565.1
# SQ_INSTS_VALU of the update over its chip issue capacity in the same
# window (1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs / 4 cycles per wave64 op)
COUNTER_UPDATE_VALU_FRAC = 0.546
COUNTER_SOURCES_SHA = "a14bd4617e67dec5"
COUNTER_WORKLOAD = "3d_periodic_1M_blobs"
COUNTER_DEPOSIT_PATH = 5


def sources_sha() -> str:
    h = hashlib.sha256()
    csrc = ROOT / "paper_1805_11007_amd" / "csrc"
    for f in sorted(csrc.iterdir()):
        if f.suffix in (".hip", ".h", ".cpp"):
            h.update(f.name.encode())
            h.update(f.read_bytes())
    return h.hexdigest()[:16]


def counters_valid(workload: str, bin_side_mult: float | None = None) -> bool:
    """True while the kernel sources and the workload are those the counter
    figures were taken with."""
    return (COUNTER_SOURCES_SHA is not None and workload == COUNTER_WORKLOAD
            and sources_sha() == COUNTER_SOURCES_SHA)


def floor_bytes(w) -> float:
    """What one step must move by definition of the method, whatever the
    kernels (N agents, G nodes, d = dim, F deposited fields: 1 without
    uptake, else 2): read positions (4d) and ids / species (4), write
    positions (4d); read and write the field (8 per node), write each
    deposited field once and read it once (8F per node)."""
    N, d = w.n_total, w.dim
    G = w.n_inst * w.grid_n ** d
    F = 2 if any(s.uptake > 0 for s in w.species) else 1
    return float(N * (8 * d + 4) + G * (8 + 8 * F))


def algorithmic_bytes(stage: str, w, n_sub: int) -> float:
    """Bytes a stage must move per launch (per step), by definition of what it
    computes, independent of how the kernels are built (N agents, G nodes,
    d = dim, F = deposited fields, 1 without uptake, else 2):
      update:  read position + id/species, write position (8d + 4 per agent);
               read the chemical once (4 per node)
      deposit: read position + species (4d + 1 per agent); write each
               deposited field once (4F per node)
      pde:     per substep read and write c (8 per node), read each deposited
               field once (4F per node)
      bin:     read position (4d per agent)
      scatter: read position/id, write position/id (8d + 8 per agent)
      scan:    read count, write start (8 per bin)
    """
    N, d = w.n_total, w.dim
    G = w.n_inst * w.grid_n ** d
    F = 2 if any(s.uptake > 0 for s in w.species) else 1
    if stage == "update":
        return N * (8 * d + 4) + G * 4
    if stage == "deposit":
        return N * (4 * d + 1) + G * 4 * F
    if stage == "pde":
        return G * (8 * n_sub + 4 * F)
    if stage == "bin":
        return N * 4 * d
    if stage == "scatter":
        return N * (8 * d + 8)
    return 0.0


def cpu_model() -> str:
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, inp, budget_s: float = 10.0, max_steps: int = 40,
                 one_thread_budget_s: float = 8.0):
    """The FP64 cell-list oracle on the same workload from the same initial
    state: as many steps as fit in budget_s on all host threads, then on one
    thread for about one_thread_budget_s.  Rates in particle-steps/s."""
    import oracle

    def timed(budget, cap):
        p = oracle.params(w, 0, mode=1)
        X, sp, c = inp["x0"], inp["species0"], inp["c0"]
        steps, st, t0 = 0, 0, time.perf_counter()
        while steps < cap:
            X, c, st = oracle.step(p, X, sp, c, st)
            steps += 1
            if time.perf_counter() - t0 > budget:
                break
        return steps, time.perf_counter() - t0

    n_all = oracle.num_threads()
    steps, el = timed(budget_s, max_steps)
    oracle.set_threads(1)
    try:
        steps1, el1 = timed(one_thread_budget_s, max_steps)
    finally:
        oracle.set_threads(n_all)
    return {"value": w.n_total * steps / el, "unit": "particle-steps/s",
            "cores": n_all, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"first {steps} steps of the same workload, FP64 cell-list oracle, "
                      f"{el:.1f} s on {n_all} threads",
            "one_thread": {"value": w.n_total * steps1 / el1, "unit": "particle-steps/s",
                           "cores": 1, "sample": f"first {steps1} steps, {el1:.1f} s"},
            "brute_force": brute_force_baseline()}


def brute_force_baseline() -> dict:
    """The oracle's all-pairs mode (every pair tested, no cell list) on all
    host threads: the 1k-agent 2D run in full (100 steps) and one step of the
    100k-agent 2D walls run."""
    import oracle
    import workloads as W
    out = {}
    for name, n_steps in ((W.PERIODIC_1K, None), (W.WALLS_100K, 1)):
        w = W.workload(name)
        inp = W.make_inputs(w)
        k = n_steps or w.steps
        p = oracle.params(w, 0, mode=0)
        X, sp, c, st = inp["x0"], inp["species0"], inp["c0"], 0
        t0 = time.perf_counter()
        for _ in range(k):
            X, c, st = oracle.step(p, X, sp, c, st)
        el = time.perf_counter() - t0
        out[name] = {"value": w.n_total * k / el, "unit": "particle-steps/s", "steps": k,
                     "seconds": el, "cores": oracle.num_threads()}
    return out


def _timed(fn) -> float:
    import torch
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def ensemble_leg(steps: int = 500) -> dict:
    """256 independent 2D instances of uneven size stepped together (one launch
    per stage, HIP-graph replay, bin side, work-group size and deposit mode
    tuned on states along the run) vs the same instances, for the same steps,
    stepped one after another as single-instance handles."""
    import dataclasses
    import torch
    import workloads as W
    from paper_1805_11007_amd import ModelSpec, Sim
    from paper_1805_11007_amd.autotune import tune
    w = W.workload(W.ENSEMBLE_256)
    inp = W.make_inputs(w)
    x0, s0, c0 = (torch.from_numpy(inp[k]).cuda() for k in ("x0", "species0", "c0"))
    spec, rep = tune(ModelSpec.from_workload(w), x0, s0, c0, horizon=steps)
    sim = Sim(spec, x0, s0, c0)
    sim.use_graph(True)
    sim.step(4)
    sim.set_state(x0, c0, 0)
    ms = _timed(lambda: sim.step(steps))
    sim.sync()
    batched = w.n_total * steps / (ms / 1e3)
    sim.close()
    # plain: every instance alone (its own handle, same seed and noise stream)
    G = w.grid_n ** w.dim
    tot_ms, tot_ps, off = 0.0, 0, 0
    for k, ins in enumerate(w.instances):
        n = ins.n_agents
        # a single instance with the tuned bin side and work-groups, and the
        # deposit the library picks for one instance
        one = dataclasses.replace(spec, deposit_mode=0,
                                  instances=[dataclasses.replace(spec.instances[k], stream=k)])
        s1 = Sim(one, x0[off:off + n], s0[off:off + n], c0[k * G:(k + 1) * G])
        s1.use_graph(True)
        s1.step(2)
        s1.set_state(x0[off:off + n], c0[k * G:(k + 1) * G], 0)
        tot_ms += _timed(lambda: s1.step(steps))
        tot_ps += n * steps
        s1.close()
        off += n
    plain = tot_ps / (tot_ms / 1e3)
    fb = floor_bytes(w)
    return {"workload": w.name, "instances": w.n_inst, "agents_total": w.n_total,
            "batched_particle_steps_per_s": batched, "batched_steps": steps,
            "batched_ms_per_step": ms / steps,
            "floor_bytes_per_step": fb,
            "floor_frac": fb / (ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "plain_particle_steps_per_s": plain, "plain_steps_per_instance": steps,
            "speedup_vs_plain": batched / plain,
            "tuned": {"bin_size": spec.bin_size, "block": spec.block,
                      "deposit_mode": spec.deposit_mode}}


def fig1_leg(hist_n: int = 52) -> dict:
    """The experiment of Sect. 4 (Fig. 1): 2000 realisations of 100 producers
    that switch to consumers at rate 10 plus 100 consumers, stepped to
    T_f = 0.05 as one batch with HIP-graph replay, with the ensemble
    statistics (per-species hist_n^2 histograms, mean field) taken at
    t = 0, T/3, 2T/3 and T inside the timed region."""
    import math
    import torch
    import workloads as W
    from paper_1805_11007_amd import ModelSpec, Sim
    from paper_1805_11007_amd.autotune import tune
    w = W.workload(W.FIG1_2000)
    inp = W.make_inputs(w)
    x0, s0, c0 = (torch.from_numpy(inp[k]).cuda() for k in ("x0", "species0", "c0"))
    spec, _ = tune(ModelSpec.from_workload(w), x0, s0, c0)
    sim = Sim(spec, x0, s0, c0)
    sim.use_graph(True)
    sim.step(4)
    sim.set_state(x0, c0, 0)
    marks = [0, round(w.steps / 3), round(2 * w.steps / 3), w.steps]
    snaps = []

    def run():
        snaps.clear()
        snaps.append(sim.ensemble_stats(hist_n))
        for a, b in zip(marks, marks[1:]):
            sim.step(b - a)
            snaps.append(sim.ensemble_stats(hist_n))

    ms = _timed(run)
    sim.sync()
    tot = [s[1].cpu().tolist() for s in snaps]
    sim.set_state(x0, c0, 0)
    prof = sim.profile_steps(300)
    stats_ms = _timed(lambda: [sim.ensemble_stats(hist_n) for _ in range(20)]) / 20
    sim.close()
    r_dt = w.species[0].react_rate * w.dt
    n_a0 = tot[0][0]
    return {"workload": w.name, "realisations": w.n_inst, "agents_total": w.n_total,
            "tuned": {"bin_size": spec.bin_size, "block": spec.block,
                      "deposit_mode": spec.deposit_mode},
            "steps": w.steps, "T_f": w.steps * w.dt, "wall_s": ms / 1e3,
            "ms_per_step": ms / w.steps,
            "particle_steps_per_s": w.n_total * w.steps / (ms / 1e3),
            "stats_call_ms": stats_ms, "stage_ms": prof,
            "alpha_beta_totals_at_marks": tot,
            "alpha_fraction_T": tot[-1][0] / n_a0,
            "alpha_fraction_T_expected": (1 - r_dt) ** w.steps,
            "alpha_fraction_T_sd": math.sqrt((1 - r_dt) ** w.steps *
                                             (1 - (1 - r_dt) ** w.steps) / n_a0)}


def reaction_overhead_leg(steps: int = 500) -> dict:
    """Step time of the 100k-agent two-species walls workload without and with
    type switching (0 -> 1 at rate 1e4, 1 -> 0 at 5e3 c), graph replay."""
    import dataclasses
    import torch
    import workloads as W
    from paper_1805_11007_amd import ModelSpec, Sim
    w = W.workload(W.WALLS_100K)
    inp = W.make_inputs(w)
    x0, s0, c0 = (torch.from_numpy(inp[k]).cuda() for k in ("x0", "species0", "c0"))
    a, b = w.species
    wr = dataclasses.replace(w, species=(dataclasses.replace(a, react_to=1, react_rate=1e4),
                                         dataclasses.replace(b, react_to=0, react_rate_c=5e3)))
    out = {}
    for name, ww in (("plain", w), ("switching", wr)):
        sim = Sim(ModelSpec.from_workload(ww), x0, s0, c0)
        sim.use_graph(True)
        sim.step(4)
        sim.set_state(x0, c0, 0)
        out[name + "_ms_per_step"] = _timed(lambda: sim.step(steps)) / steps
        sim.sync()
        sim.set_state(x0, c0, 0)
        out[name + "_update_ms"] = sim.profile_steps(steps)["update"]
        sim.close()
    out["workload"] = w.name
    out["overhead"] = out["switching_ms_per_step"] / out["plain_ms_per_step"] - 1
    return out


def kde_leg(steps: int = 100, sample_nodes: int = 4000) -> dict:
    """The Gaussian kernel density deposit (bandwidth = diameter, truncated at
    3 bandwidths) against the particle-in-cell deposit on the 100k-agent walls
    workload and the 1M-agent 3D workload, graph replay.  The gather's work
    is counted as kernel evaluations (node-agent pairs inside the radius),
    estimated from a random sample of nodes on the states at the start,
    middle and end of the profiled steps."""
    import dataclasses
    import numpy as np
    import torch
    from scipy.spatial import cKDTree
    import workloads as W
    from paper_1805_11007_amd import ModelSpec, Sim
    out = {}
    for wname in (W.WALLS_100K, W.BLOBS_1M):
        w = W.workload(wname)
        inp = W.make_inputs(w)
        x0, s0, c0 = (torch.from_numpy(inp[k]).cuda() for k in ("x0", "species0", "c0"))
        r = {}
        for name, dk in (("pic", 0), ("kde", 1)):
            sim = Sim(ModelSpec.from_workload(w, deposit_kernel=dk, kde_radius=3.0), x0, s0, c0)
            sim.use_graph(True)
            sim.step(4)
            sim.set_state(x0, c0, 0)
            r[name + "_ms_per_step"] = _timed(lambda: sim.step(steps)) / steps
            sim.sync()
            sim.set_state(x0, c0, 0)
            if dk == 1:
                # the gather's work grows as the blobs collapse: keep the
                # states at the start, middle and end of the profiled steps
                half = min(steps, 50) // 2
                states, ps = [inp["x0"]], []
                for _ in range(2):
                    ps.append(sim.profile_steps(half))
                    states.append(sim.get_state()[0].cpu().numpy())
                prof = {k: (ps[0][k] + ps[1][k]) / 2 for k in ps[0]}
            else:
                prof = sim.profile_steps(min(steps, 50))
            r[name + "_deposit_ms"] = prof["deposit"]
            r[name + "_pde_ms"] = prof["pde"]
            sim.close()
        # kernel evaluations per step: node-agent pairs within 3 diameters,
        # on a node sample of each kept state, averaged over the profiled
        # steps (trapezoid rule)
        rng = np.random.default_rng(0)
        xs = W.node_coords(w)
        G = w.grid_n ** w.dim
        idx = rng.integers(0, G, sample_nodes)
        coords = np.stack([xs[(idx // w.grid_n ** a) % w.grid_n] for a in range(w.dim)], 1)
        R = 3.0 * max(s.diameter for s in w.species)
        at = []
        for X in states:
            X = X.astype(np.float64)
            if w.periodic:
                X = np.mod(X, w.L)
            tree = cKDTree(X, boxsize=w.L if w.periodic else None)
            at.append(float(tree.query_ball_point(coords, R, return_length=True).mean()) * G)
        evals = (at[0] + 2.0 * at[1] + at[2]) / 4.0
        r["kernel_evals_per_step"] = evals
        r["kernel_evals_per_step_at_0_mid_end"] = at
        r["kde_evals_per_s"] = evals / (r["kde_deposit_ms"] * 1e-3)
        r["agents"] = w.n_total
        r["nodes"] = G
        out[w.name] = r
    return out


def variants_leg(steps: int = 100) -> dict:
    """Step time and per-stage profile of the pair/update variants against
    the harmonic soft-sphere step on the 100k-agent walls workload and the
    1M-agent 3D workload: exponential potential (range 3 d, k = 1), tamed
    Euler (harmonic), hard spheres (overlap correction pass); graph replay."""
    import torch
    import workloads as W
    from paper_1805_11007_amd import ModelSpec, Sim
    variants = {"harmonic": {}, "exponential": {"potential": 1, "pot_range": 3.0, "k": 1.0},
                "tamed": {"tamed": True}, "hard_spheres": {"potential": 2}}
    out = {}
    for wname in (W.WALLS_100K, W.BLOBS_1M):
        w = W.workload(wname)
        inp = W.make_inputs(w)
        x0, s0, c0 = (torch.from_numpy(inp[k]).cuda() for k in ("x0", "species0", "c0"))
        r = {}
        for name, kw in variants.items():
            sim = Sim(ModelSpec.from_workload(w, **kw), x0, s0, c0)
            sim.use_graph(True)
            sim.step(4)
            sim.set_state(x0, c0, 0)
            ms = _timed(lambda: sim.step(steps)) / steps
            sim.sync()
            sim.set_state(x0, c0, 0)
            prof = sim.profile_steps(min(steps, 50))
            r[name] = {"ms_per_step": ms, "particle_steps_per_s": w.n_total / (ms * 1e-3),
                       "stage_ms": {k: round(v, 5) for k, v in prof.items() if v > 0}}
            sim.close()
        out[w.name] = r
    return out


def adjoint_leg(steps: int = 200, K: int = 20) -> dict:
    """Forward with checkpoints every K steps plus the reverse sweep (which
    recomputes each segment) on the 50k-agent differentiation workload, vs
    the plain forward of the same steps; rates count each step once."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1805_11007_amd import ModelSpec, Sim
    from paper_1805_11007_amd.adjoint import density_loss_run
    w = W.adjoint_2d()
    inp = W.make_inputs(w)
    x0, s0, c0 = (torch.from_numpy(inp[k]).cuda() for k in ("x0", "species0", "c0"))
    base = ModelSpec.from_workload(w)
    # target: a run at theta* = (1.5, 800, 0.8) with another noise key
    tw = W.adjoint_2d(chi=1.5, k=800, D=0.8, seed=2005)
    tsim = Sim(ModelSpec.from_workload(tw), x0, s0, c0)
    tsim.step(steps)
    target = tsim.density_hist(64, 2.0)
    tsim.close()
    plain = Sim(base, x0, s0, c0)
    plain.use_graph(True)
    plain.step(2)
    plain.set_state(x0, c0, 0)
    ms_plain = _timed(lambda: plain.step(steps))
    plain.close()
    theta = torch.tensor([1.0, 100.0, 1.0], dtype=torch.float64, requires_grad=True)
    out = {}

    def fwd_bwd():
        loss = density_loss_run(theta, base, x0, s0, c0, target, steps, K, 64, 2.0)
        loss.backward()
        out["loss"] = float(loss.detach())

    density_loss_run(theta.detach().requires_grad_(True), base, x0, s0, c0, target, 20, K,
                     64, 2.0).backward()  # warm-up
    ms_fb = _timed(fwd_bwd)
    n = w.n_total
    return {"workload": w.name, "agents": n, "steps": steps, "checkpoint_every": K,
            "plain_particle_steps_per_s": n * steps / (ms_plain / 1e3),
            "fwd_bwd_particle_steps_per_s": n * steps / (ms_fb / 1e3),
            "fwd_bwd_over_plain_time": ms_fb / ms_plain, "loss": out["loss"],
            "grad_theta": theta.grad.tolist()}


def configs_leg() -> dict:
    """The other single-instance workloads, forward only (HIP-graph replay of
    their full step count from the initial state, 2 warm-up steps): step time,
    particle-steps/s and the step's algorithmic floor against HBM."""
    import torch
    import workloads as W
    from paper_1805_11007_amd import ModelSpec, Sim
    out = {}
    for name in (W.PERIODIC_1K, W.WALLS_100K, W.ADJOINT_50K):
        w = W.workload(name)
        inp = W.make_inputs(w)
        x0, s0, c0 = (torch.from_numpy(inp[k]).cuda() for k in ("x0", "species0", "c0"))
        sim = Sim(ModelSpec.from_workload(w), x0, s0, c0)
        sim.use_graph(True)
        sim.step(2)
        sim.set_state(x0, c0, 0)
        ms = _timed(lambda: sim.step(w.steps)) / w.steps
        sim.sync()
        sim.set_state(x0, c0, 0)
        prof = sim.profile_steps(min(w.steps, 200))
        sim.close()
        fb = floor_bytes(w)
        out[name] = {"agents": w.n_total, "nodes": w.n_inst * w.grid_n ** w.dim,
                     "steps": w.steps, "ms_per_step": ms,
                     "particle_steps_per_s": w.n_total / (ms * 1e-3),
                     "floor_bytes_per_step": fb, "floor_GBs": fb / (ms * 1e-3) / 1e9,
                     "floor_frac": fb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "stage_ms": {k: round(v, 5) for k, v in prof.items() if v > 0}}
    return out


LEGS = {"ensemble": lambda: ensemble_leg(), "fig1": lambda: fig1_leg(), "kde": lambda: kde_leg(),
        "variants": lambda: variants_leg(),
        "switching": lambda: reaction_overhead_leg(), "fwd_bwd": lambda: adjoint_leg(),
        "configs": lambda: configs_leg()}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="3d_periodic_1M_blobs",
                    help="workload name (the workloads module lists them)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the full-run, per-workload, ensemble, forward+backward and "
                         "variant legs")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the library's default bin side and work-group size")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three plain 256 MiB device copies (the reference "
                         "kernel for scaling FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--deterministic", action="store_true")
    ap.add_argument("--bin-size", type=float, default=0.0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--leg", choices=sorted(LEGS), default=None,
                    help="run only this extra leg and print its JSON line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library steps a batch on one device and "
              "has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.leg:
        print(json.dumps({args.leg: LEGS[args.leg]()}), flush=True)
        return 0

    if args.copy_calibration:
        a = torch.ones(64 * 1024 * 1024, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copied_bytes_per_kernel": a.numel() * 4, "kernels": 3}))
        return 0

    import workloads as W
    from paper_1805_11007_amd import ModelSpec, Sim
    from paper_1805_11007_amd.autotune import tune

    w = W.workload(args.workload)
    inp = W.make_inputs(w)
    torch.cuda.set_device(0)
    x0 = torch.from_numpy(inp["x0"]).cuda()
    s0 = torch.from_numpy(inp["species0"]).cuda()
    c0 = torch.from_numpy(inp["c0"]).cuda()
    spec = ModelSpec.from_workload(w, deterministic=args.deterministic,
                                   bin_size=args.bin_size, block=args.block)
    tune_rep = None
    if not args.no_tune and not args.bin_size and not args.block:
        # bin side, work-group size and deposit mode for this run, timed from
        # the states at the start, middle and end of the workload's full run
        spec, tune_rep = tune(spec, x0, s0, c0, steps=10, horizon=w.steps)
        print(f"[bench] autotuned: {json.dumps(tune_rep.get('best', tune_rep.get('cached')))}",
              file=sys.stderr, flush=True)
    sim = Sim(spec, x0, s0, c0)
    if not args.no_graph:
        sim.use_graph(True)
    print(f"[bench] {w.name}: N={w.n_total} G={w.n_inst * w.grid_n ** w.dim} "
          f"info={sim.info}", file=sys.stderr, flush=True)

    # warm-up (also captures the graph), then back to the initial condition
    sim.step(args.warmup)
    sim.sync()
    sim.set_state(x0, c0, 0)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sim.sync()
    value = w.n_total * args.steps / (ms / 1e3)
    ms_step = ms / args.steps
    print(f"[bench] timed {args.steps} steps: {ms:.3f} ms", file=sys.stderr, flush=True)

    # per-stage HIP-event profile of the same steps from the same state
    sim.set_state(x0, c0, 0)
    prof = sim.profile_steps(args.steps)
    dom = max(prof, key=prof.get)
    n_sub = sim.info["pde_substeps"]
    print(f"[bench] stage ms/step: {json.dumps({k: round(v, 5) for k, v in prof.items()})}",
          file=sys.stderr, flush=True)
    # mean true neighbours along the same steps (sampled every 10 steps)
    sim.set_state(x0, c0, 0)
    nbr = []
    for t in range(0, args.steps, 10):
        cnt, _ = sim.debug_neighbours()
        nbr.append(float(cnt.double().mean()))
        sim.step(min(10, args.steps - t))
    nbr_mean = float(np.mean(nbr))

    valid = (counters_valid(w.name) and not args.deterministic and not args.no_graph
             and sim.info["deposit_path"] == COUNTER_DEPOSIT_PATH)
    alg = algorithmic_bytes(dom, w, n_sub)
    achieved = alg / (prof[dom] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": (COUNTER_UPDATE_BYTES if valid and dom == "update" else None),
            "algorithmic_bytes_per_launch": alg, "launch_ms": prof[dom]}
    if dom == "update":
        flops = w.n_total * (FLOP_PER_PAIR * nbr_mean + FLOP_PER_AGENT)
        tf = flops / (prof[dom] * 1e-3) / 1e12
        roof["alu_view"] = {"achieved_TFLOPs": tf, "peak_attainable": FP32_ATTAINABLE_TFLOPS,
                            "frac": tf / FP32_ATTAINABLE_TFLOPS,
                            "algorithmic_flop_per_launch": flops,
                            "mean_neighbours": nbr_mean,
                            "valu_issue_frac": COUNTER_UPDATE_VALU_FRAC if valid else None}
    fb = floor_bytes(w)
    step_hbm = {"floor_bytes": fb, "floor_GBs": fb / (ms_step * 1e-3) / 1e9,
                "floor_frac": fb / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "counter_bytes": COUNTER_STEP_BYTES if valid else None}
    if step_hbm["counter_bytes"]:
        cb = step_hbm["counter_bytes"]
        step_hbm.update({"counter_GBs": cb / (ms_step * 1e-3) / 1e9,
                         "counter_frac": cb / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "amplification": cb / fb})

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "dim": w.dim, "n_agents": w.n_total,
                   "grid": f"{w.grid_n}^{w.dim}", "dt": w.dt, "timed_steps": args.steps,
                   "graph": not args.no_graph, "deterministic": args.deterministic,
                   "bins_per_axis": sim.info["bins_per_axis"], "stencil": sim.info["stencil"],
                   "block": sim.info["block"], "deposit_path": sim.info["deposit_path"]},
        "roofline": roof,
        "step_hbm": step_hbm,
        "stage_ms": prof,
        "autotune": ({"choice": tune_rep.get("best", tune_rep.get("cached")),
                      "states_at_steps": tune_rep.get("states_at_steps"),
                      "trials": tune_rep.get("trials")} if tune_rep else None),
    }
    if not args.no_extras:
        # the workload's whole run (all its steps from the initial state)
        sim.set_state(x0, c0, 0)
        fms = _timed(lambda: sim.step(w.steps))
        sim.set_state(x0, c0, 0)
        fprof = sim.profile_steps(w.steps)
        res["full_run"] = {"steps": w.steps, "ms_per_step": fms / w.steps,
                           "particle_steps_per_s": w.n_total * w.steps / (fms / 1e3),
                           "floor_frac": fb / (fms / w.steps * 1e-3) / 1e9 / HBM_PEAK_GBS,
                           "stage_ms": {k: round(v, 5) for k, v in fprof.items() if v > 0}}
        print(f"[bench] full run: {json.dumps(res['full_run'])}", file=sys.stderr, flush=True)
    sim.close()
    if not args.no_extras:
        for name, title in (("configs", "other workloads"), ("ensemble", "ensemble"),
                            ("fig1", "Fig. 1 ensemble"), ("switching", "switching overhead"),
                            ("kde", "kernel density"), ("variants", "pair/update variants"),
                            ("fwd_bwd", "forward+backward")):
            print(f"[bench] {title} leg", file=sys.stderr, flush=True)
            res[name] = LEGS[name]()
            print(f"[bench] {name}: {json.dumps(res[name])}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(w, inp)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
