"""Autotuner for the step's launch choices.

It searches the cell-list bin side (as a multiple of the largest contact
distance: 1.0 selects the 3^dim stencil, >= 2.0 the 2^dim half-bin stencil)
and the work-group size of the agent kernels, then, with the best of those,
the deposit mode (LDS-aggregated, direct atomics, or deposit + PDE fused per
instance where an instance's sums fit in LDS).  It times a few steps of each
candidate on the caller's own initial state, with HIP-graph replay, and
returns the fastest.  Results are cached in a JSON file keyed by device
name, dimension, agent-count bucket, instance count, grid size and boundary
type, so later runs of the same shape reuse them without timing.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os
from pathlib import Path

import torch

from .sim import ModelSpec, Sim

CANDIDATE_BINS = (1.0, 1.25, 2.0)
CANDIDATE_BLOCKS = (128, 256, 512)
CANDIDATE_DEPOSIT = (1, 2, 3)


def cache_path() -> Path:
    p = os.environ.get("PC_AUTOTUNE_CACHE")
    if p:
        return Path(p)
    return Path.home() / ".cache" / "paper_1805_11007_amd" / "autotune.json"


def shape_key(spec: ModelSpec) -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    n = spec.n_total
    bucket = 2 ** round(math.log2(max(n, 1)))
    return (f"{dev}|d{spec.dim}|N~{bucket}|inst{len(spec.instances)}|g{spec.grid_n}|"
            f"{'per' if spec.periodic else 'wall'}|ns{len(spec.species)}")


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


def time_steps(spec: ModelSpec, x0, s0, c0, steps: int, warmup: int = 2) -> float:
    """Mean milliseconds per step of `steps` graph-replayed steps."""
    sim = Sim(spec, x0, s0, c0)
    sim.use_graph(True)
    sim.step(warmup)
    sim.set_state(x0, c0, 0)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    sim.close()
    return e0.elapsed_time(e1) / steps


def tune(spec: ModelSpec, x0, s0, c0, steps: int = 10, use_cache: bool = True,
         bins=CANDIDATE_BINS, blocks=CANDIDATE_BLOCKS,
         deposit_modes=CANDIDATE_DEPOSIT) -> tuple[ModelSpec, dict]:
    """Return (spec with the fastest bin_size, block and deposit mode, report)."""
    key = shape_key(spec)
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
    trials = []
    for bm in bins:
        side = bm * cut * (1 + 2e-4)
        if spec.L / side < 3:
            continue
        for blk in blocks:
            cand = dataclasses.replace(spec, bin_size=side, block=blk)
            try:
                ms = time_steps(cand, x0, s0, c0, steps)
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
            ms = time_steps(cand, x0, s0, c0, steps)
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
    return tuned, {"trials": trials, "best": best}
