"""Autotuner for the step's launch choices.

It searches the cell-list bin side (as a multiple of the largest contact
distance: below 2.0 the 3^dim stencil, from 2.0 the 2^dim half-bin stencil;
the paper's default of about ten agents per bin with a tunable side, Sect.
3.1) and the work-group size of the agent kernels, then, with the best of
those, the deposit mode (LDS-aggregated, direct atomics, deposit + PDE
fused per instance where an instance's sums fit in LDS, or owner-computes
node slabs).  Each candidate
is timed with HIP-graph replay over a few steps from each of a set of
representative states: the caller's initial state alone, or, with a
horizon, the states at the start, middle and end of a run of that many
steps (a clustering run costs several times more per step at its end than
at its start).  The fastest mean wins.  Results are cached in a JSON file
keyed by device name, dimension, agent-count bucket, instance count, grid
size, boundary type, species count and horizon, so later runs of the same
shape reuse them without timing.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os
from pathlib import Path

import torch

from .sim import ModelSpec, Sim

CANDIDATE_BINS = (1.0, 1.25, 1.5, 2.0)
CANDIDATE_BLOCKS = (64, 128, 256)
CANDIDATE_DEPOSIT = (1, 2, 3, 4)


def cache_path() -> Path:
    p = os.environ.get("PC_AUTOTUNE_CACHE")
    if p:
        return Path(p)
    return Path.home() / ".cache" / "paper_1805_11007_amd" / "autotune.json"


def device_key() -> str:
    """The device's ISA and compute-unit count (its marketing name is not
    always available, e.g. under a profiler)."""
    if not torch.cuda.is_available():
        return "cpu"
    pr = torch.cuda.get_device_properties(0)
    arch = getattr(pr, "gcnArchName", "") or torch.cuda.get_device_name(0) or "gpu"
    return f"{arch.split(':')[0]}x{pr.multi_processor_count}"


def shape_key(spec: ModelSpec, horizon: int = 0) -> str:
    dev = device_key()
    n = spec.n_total
    bucket = 2 ** round(math.log2(max(n, 1)))
    return (f"{dev}|d{spec.dim}|N~{bucket}|inst{len(spec.instances)}|g{spec.grid_n}|"
            f"{'per' if spec.periodic else 'wall'}|ns{len(spec.species)}|T{horizon}")


def _load() -> dict:
    try:
        return json.loads(cache_path().read_text())
    except (OSError, ValueError):
        return {}


def _store(d: dict) -> None:
    p = cache_path()
    try:
        p.parent.mkdir(parents=True, exist_ok=True)
        tmp = p.with_suffix(".tmp%d" % os.getpid())
        tmp.write_text(json.dumps(d, indent=1, sort_keys=True))
        os.replace(tmp, p)
    except OSError:
        pass  # a read-only home only disables the cache


def representative_states(spec: ModelSpec, x0, s0, c0, horizon: int, steps: int) -> list:
    """States (x, c, step) at the start, middle and end of a run of `horizon`
    steps of `spec` from the given initial state (the end one `steps` before
    the horizon, so that timing from it stays inside the run)."""
    marks = sorted({0, max(0, horizon // 2), max(0, horizon - steps)})
    sim = Sim(spec, x0, s0, c0)
    sim.use_graph(True)
    out, done = [], 0
    for m in marks:
        sim.step(m - done)
        done = m
        out.append(sim.get_state())
    sim.close()
    return out


def time_steps(spec: ModelSpec, x0, s0, c0, steps: int, warmup: int = 2,
               states: list | None = None) -> float:
    """Mean milliseconds per step of `steps` graph-replayed steps, from the
    initial state or averaged over the given (x, c, step) states."""
    sim = Sim(spec, x0, s0, c0)
    sim.use_graph(True)
    sim.step(warmup)
    stream = torch.cuda.current_stream()
    tot = 0.0
    for x, c, st in (states or [(x0, c0, 0)]):
        sim.set_state(x, c, st)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        sim.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        tot += e0.elapsed_time(e1) / steps
    sim.close()
    return tot / len(states or [None])


def tune(spec: ModelSpec, x0, s0, c0, steps: int = 10, use_cache: bool = True,
         bins=CANDIDATE_BINS, blocks=CANDIDATE_BLOCKS,
         deposit_modes=CANDIDATE_DEPOSIT, horizon: int = 0) -> tuple[ModelSpec, dict]:
    """Return (spec with the fastest bin_size, block and deposit mode, report).
    With horizon > 0 every candidate is timed from the states at the start,
    middle and end of a horizon-step run of the given spec."""
    key = shape_key(spec, horizon)
    cache = _load() if use_cache else {}
    cut = max(s.diameter for s in spec.species)
    if key in cache:
        c = cache[key]
        return dataclasses.replace(spec, bin_size=c["bin_mult"] * cut * (1 + 2e-4) if
                                   c["bin_mult"] else 0.0, block=c["block"],
                                   deposit_mode=c.get("deposit_mode", 0)), {"cached": c}
    x0 = x0.cuda()
    s0 = s0.cuda()
    c0 = c0.cuda()
    states = representative_states(spec, x0, s0, c0, horizon, steps) if horizon > 0 else None
    trials = []
    for bm in bins:
        side = bm * cut * (1 + 2e-4)
        if spec.L / side < 3:
            continue
        for blk in blocks:
            cand = dataclasses.replace(spec, bin_size=side, block=blk)
            try:
                ms = time_steps(cand, x0, s0, c0, steps, states=states)
            except Exception as e:  # an invalid candidate (e.g. too many bins) is skipped
                trials.append({"bin_mult": bm, "block": blk, "error": str(e)})
                continue
            trials.append({"bin_mult": bm, "block": blk, "ms_per_step": ms})
    ok = [t for t in trials if "ms_per_step" in t]
    if not ok:
        return spec, {"trials": trials}
    best = dict(min(ok, key=lambda t: t["ms_per_step"]), deposit_mode=spec.deposit_mode)
    side = best["bin_mult"] * cut * (1 + 2e-4)
    for dm in deposit_modes:
        if dm == spec.deposit_mode:
            continue
        cand = dataclasses.replace(spec, bin_size=side, block=best["block"], deposit_mode=dm)
        try:
            ms = time_steps(cand, x0, s0, c0, steps, states=states)
        except Exception as e:  # e.g. per-instance sums that do not fit in LDS
            trials.append({"deposit_mode": dm, "error": str(e)})
            continue
        trials.append({"bin_mult": best["bin_mult"], "block": best["block"], "deposit_mode": dm,
                       "ms_per_step": ms})
        if ms < best["ms_per_step"]:
            best = {"bin_mult": best["bin_mult"], "block": best["block"], "deposit_mode": dm,
                    "ms_per_step": ms}
    if use_cache:
        cache[key] = {"bin_mult": best["bin_mult"], "block": best["block"],
                      "deposit_mode": best["deposit_mode"], "ms_per_step": best["ms_per_step"]}
        _store(cache)
    tuned = dataclasses.replace(spec, bin_size=side, block=best["block"],
                                deposit_mode=best["deposit_mode"])
    return tuned, {"trials": trials, "best": best,
                   "states_at_steps": [st for _, _, st in states] if states else [0]}
