"""Seeded synthetic workloads for the hybrid chemotaxis step.

This module is shared by the tests, the benchmark and the CPU oracle's
drivers.  It only *describes* workloads (parameters and sizes) and draws
their initial conditions; it contains none of the method's arithmetic
(no forces, noise, interpolation, deposit or PDE update).  Every array it
returns is the exact input given to both the GPU library and the oracle.

The paper runs its own simulations only (no public dataset); the six
workloads below stand in for them (``workload(name)``):

* ``2d_periodic_1k``           2D periodic, 1,000 agents, 64^2 grid (parity case)
* ``2d_walls_100k``            2D reflecting walls, 100,000 agents in two species,
  512^2 grid
* ``3d_periodic_1M_blobs``     3D periodic, 1,000,000 agents in 8 Gaussian blobs,
  128^3 grid
* ``2d_ensemble_256``          256 independent 2D instances of uneven size, 128^2
  grids
* ``2d_periodic_50k_adjoint``  2D periodic, 50,000 agents (producers /
  consumers), 256^2 grid; ``adjoint_2d`` sets its parameters
* ``2d_walls_fig1_2000x200``   2000 realisations of the experiment of Sect. 4
  (Fig. 1): 100 producers that switch to consumers plus 100 consumers each,
  reflecting walls, 52^2 grid; ``fig1_walls_2d`` sets its size

Initial conditions follow one recipe: a numpy ``PCG64`` generator with the
workload's own seed (1001 ... 1006 in the order above) draws everything in
float64, which is then rounded to float32 (positions) so that both sides
start from identical float32 arrays.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field, replace
from typing import List, Sequence, Tuple

import numpy as np

__all__ = ["Species", "Instance", "Workload", "workload", "adjoint_2d", "fig1_walls_2d",
           "scaled", "make_inputs", "node_coords", "NAMES", "PERIODIC_1K", "WALLS_100K",
           "BLOBS_1M", "ENSEMBLE_256", "ADJOINT_50K", "FIG1_2000"]

PERIODIC_1K = "2d_periodic_1k"
WALLS_100K = "2d_walls_100k"
BLOBS_1M = "3d_periodic_1M_blobs"
ENSEMBLE_256 = "2d_ensemble_256"
ADJOINT_50K = "2d_periodic_50k_adjoint"
FIG1_2000 = "2d_walls_fig1_2000x200"
NAMES = (PERIODIC_1K, WALLS_100K, BLOBS_1M, ENSEMBLE_256, ADJOINT_50K, FIG1_2000)


@dataclass(frozen=True)
class Species:
    """One agent species (the paper's cell "type", Sect. 2)."""
    diameter: float   # interaction range; contact distance is the mean of two diameters
    D: float          # diffusion coefficient (eq. sde_alpha / sde_beta)
    chi: float        # chemotactic sensitivity (eq. sde_beta); 0 = no drift
    source: float     # secretion rate k_alpha (eq. pde_c)
    uptake: float     # consumption rate k_beta (eq. pde_c)
    react_to: int = -1        # type this species switches to (eq. Chemo_reactions); -1 none
    react_rate: float = 0.0   # switching rate: react_rate + react_rate_c * c(X)
    react_rate_c: float = 0.0


@dataclass(frozen=True)
class Instance:
    """One independent realisation: its size, its noise key and chi scale."""
    n_agents: int
    seed: int
    chi_scale: float = 1.0
    stream: int = -1   # noise stream index; -1: the instance's position in the list


@dataclass(frozen=True)
class Workload:
    name: str
    dim: int
    periodic: bool
    L: float
    grid_n: int
    dt: float
    k: float                 # harmonic repulsion stiffness, F = k (d - r) r_hat
    D_c: float               # chemical diffusivity
    gamma: float             # chemical decay rate
    steps: int
    species: Tuple[Species, ...]
    instances: Tuple[Instance, ...]
    pde_substeps: int = 0    # 0 = choose the smallest stable count
    layout: str = "uniform"  # "uniform" | "blobs" | "centre_uniform"
    species_rule: str = "single"  # "single" | "halves" (id >= N/2 -> species 1)
    c0: str = "sin"          # "sin": prod sin(2 pi x) + 1 ; "cos": prod cos(pi x) + 1
    gen_seed: int = 1000
    deposit_kernel: int = 0  # 0: particle-in-cell ; 1: Gaussian kernel density (Sect. 2.3)
    kde_radius: float = 3.0  # kernel truncation radius in bandwidths
    potential: int = 0       # 0 harmonic ; 1 exponential k exp(-r/d) ; 2 hard spheres
    tamed: bool = False      # tamed Euler pair drift (eq. sde_ETamed)
    pot_range: float = 3.0   # exponential potential cut at pot_range * d

    @property
    def n_total(self) -> int:
        return sum(i.n_agents for i in self.instances)

    @property
    def n_inst(self) -> int:
        return len(self.instances)

    @property
    def n_nodes(self) -> int:
        return self.grid_n ** self.dim


def _one_species() -> Tuple[Species, ...]:
    return (Species(diameter=0.01, D=1.0, chi=1.0, source=1.0, uptake=0.0),)


def workload(name: str) -> Workload:
    """One of the six workloads by name (sizes and parameters as listed in
    the module docstring)."""
    if name == PERIODIC_1K:
        return Workload(PERIODIC_1K, 2, True, 1.0, 64, 1e-5, 100.0, 1.0, 0.1, 100,
                        _one_species(), (Instance(1000, 1001),), gen_seed=1001)
    if name == WALLS_100K:
        sp = (Species(0.002, 1.0, 0.0, 1.0, 0.0), Species(0.003, 0.5, 2.0, 0.0, 1.0))
        return Workload(WALLS_100K, 2, False, 1.0, 512, 1e-6, 1000.0, 1.0, 0.1, 1000,
                        sp, (Instance(100_000, 1002),), species_rule="halves", c0="cos",
                        gen_seed=1002)
    if name == BLOBS_1M:
        sp = (Species(0.004, 1.0, 1.0, 1.0, 0.0),)
        return Workload(BLOBS_1M, 3, True, 1.0, 128, 1e-7, 1000.0, 1.0, 0.1,
                        200, sp, (Instance(1_000_000, 1003),), layout="blobs", gen_seed=1003)
    if name == ENSEMBLE_256:
        rng = np.random.Generator(np.random.PCG64(1004))
        n_i = np.rint(np.exp(rng.uniform(math.log(500), math.log(20000), 256))).astype(int)
        chi = rng.uniform(0.0, 3.0, 256)
        seeds = rng.integers(0, 2**63, 256, dtype=np.int64)
        inst = tuple(Instance(int(a), int(s), float(c)) for a, s, c in zip(n_i, seeds, chi))
        return Workload(ENSEMBLE_256, 2, True, 1.0, 128, 1e-5, 100.0, 1.0, 0.1, 500,
                        _one_species(), inst, gen_seed=1004)
    if name == ADJOINT_50K:
        return adjoint_2d()
    if name == FIG1_2000:
        return fig1_walls_2d()
    raise ValueError(f"no workload {name!r}")


def fig1_walls_2d(n_real: int = 2000, chi: float = 10.0, seed: int = 1006) -> Workload:
    """The experiment of Sect. 4 with the parameters of its Fig. 1 caption:
    N_alpha(0) = N_beta(0) = 100, diameter 0.02, r_alpha = 10, r_beta = 0,
    D_alpha = 0.1, D_beta = 1, D_c = 1, k_alpha = 0.1, k_beta = 0.03,
    dt = (0.23 * 0.02)^2 / (4 D_beta), N_c = 52, T_f = 0.05.  The caption
    leaves chi, gamma, the repulsion strength and the initial profiles open:
    chi = 10, gamma = 0, k = 1e4 (k dt = 0.05), alpha agents from a Gaussian
    of width 0.1 at the centre, beta agents uniform, c0 = 0."""
    dt = (0.23 * 0.02) ** 2 / 4.0
    sp = (Species(0.02, 0.1, 0.0, 0.1, 0.0, react_to=1, react_rate=10.0),
          Species(0.02, 1.0, chi, 0.0, 0.03))
    rng = np.random.Generator(np.random.PCG64(seed))
    seeds = rng.integers(0, 2**63, n_real, dtype=np.int64)
    inst = tuple(Instance(200, int(s)) for s in seeds)
    return Workload(FIG1_2000 if n_real == 2000 else f"2d_walls_fig1_{n_real}x200", 2, False, 1.0, 52, dt, 1e4, 1.0, 0.0,
                    int(round(0.05 / dt)), sp, inst, layout="centre_uniform",
                    species_rule="halves", c0="zero", gen_seed=seed)


def adjoint_2d(chi: float = 1.0, k: float = 100.0, D: float = 1.0, seed: int = 1005) -> Workload:
    """Differentiation workload: producers (species 0) and consumers (species 1)."""
    sp = (Species(0.01, D, 0.0, 1.0, 0.0), Species(0.01, D, chi, 0.0, 1.0))
    return Workload(ADJOINT_50K, 2, True, 1.0, 256, 1e-5, k, 1.0, 0.1, 200,
                    sp, (Instance(50_000, seed),), pde_substeps=3, species_rule="halves",
                    gen_seed=1005)



def scaled(w: Workload, n_agents: int | Sequence[int] | None = None,
           grid_n: int | None = None, steps: int | None = None, **kw) -> Workload:
    """A smaller copy of a workload with the same structure (for parity tests)."""
    inst = w.instances
    if n_agents is not None:
        if isinstance(n_agents, int):
            n_agents = [n_agents] * len(inst)
        n_agents = list(n_agents)
        if len(n_agents) != len(inst):
            inst = tuple(Instance(int(n), inst[i % len(inst)].seed + i // len(inst),
                                  inst[i % len(inst)].chi_scale)
                         for i, n in enumerate(n_agents))
        else:
            inst = tuple(replace(i, n_agents=int(n)) for i, n in zip(inst, n_agents))
    return replace(w, instances=inst, grid_n=grid_n or w.grid_n,
                   steps=w.steps if steps is None else steps, **kw)


def node_coords(w: Workload) -> np.ndarray:
    """1D node coordinates used to draw the initial chemical field.

    Periodic grids put N_c nodes at i*L/N_c; wall grids put N_c nodes at
    i*L/(N_c-1), on both walls.
    """
    n = w.grid_n
    h = w.L / n if w.periodic else w.L / (n - 1)
    return np.arange(n, dtype=np.float64) * h


def _f32_in_box(x: np.ndarray, w: Workload) -> np.ndarray:
    x32 = x.astype(np.float32)
    if w.periodic:
        # rounding can carry a value just below L up to L; keep [0, L)
        x32[x32 >= np.float32(w.L)] = np.float32(0.0)
        x32[x32 < 0] = np.float32(0.0)
    else:
        np.clip(x32, np.float32(0.0), np.float32(w.L), out=x32)
    return x32


def _positions(w: Workload, n: int, rng: np.random.Generator) -> np.ndarray:
    d = w.dim
    if w.layout == "uniform":
        x = rng.uniform(0.0, w.L, size=(n, d))
    elif w.layout == "blobs":
        centres = rng.uniform(0.0, w.L, size=(8, d))
        z = rng.standard_normal(size=(n, d))
        blob = np.arange(n) % 8
        x = np.mod(centres[blob] + 0.05 * w.L * z, w.L)
    elif w.layout == "centre_uniform":
        # first half (species 0 under the "halves" rule): Gaussian of width
        # 0.1 L at the centre, clipped to the box; second half uniform
        h = n // 2
        x = np.empty((n, d))
        x[:h] = np.clip(0.5 * w.L + 0.1 * w.L * rng.standard_normal(size=(h, d)), 0.0, w.L)
        x[h:] = rng.uniform(0.0, w.L, size=(n - h, d))
    else:
        raise ValueError(w.layout)
    return _f32_in_box(x, w)


def _field(w: Workload) -> np.ndarray:
    xs = node_coords(w)
    grids = np.meshgrid(*([xs] * w.dim), indexing="ij")  # grids[a] varies along axis a
    if w.c0 == "sin":
        f = np.ones_like(grids[0])
        for g in grids:
            f = f * np.sin(2 * np.pi * g / w.L)
        f = f + 1.0
    elif w.c0 == "cos":
        f = np.ones_like(grids[0])
        for g in grids:
            f = f * np.cos(np.pi * g / w.L)
        f = f + 1.0
    elif w.c0 == "zero":
        f = np.zeros_like(grids[0])
    else:
        raise ValueError(w.c0)
    # storage order: x fastest, i.e. C order [z][y][x] -> transpose the ij grid
    return np.ascontiguousarray(f.T).astype(np.float32).reshape(-1)


def make_inputs(w: Workload) -> dict:
    """Initial state of every instance, concatenated instance-major.

    Returns ``x0`` (float32, sum(N) x dim, id order within each instance),
    ``species0`` (uint8, sum(N)) and ``c0`` (float32, n_inst x grid_n^dim,
    x fastest).
    """
    rng = np.random.Generator(np.random.PCG64(w.gen_seed))
    xs, ss = [], []
    for inst in w.instances:
        n = inst.n_agents
        xs.append(_positions(w, n, rng))
        if w.species_rule == "single":
            ss.append(np.zeros(n, np.uint8))
        elif w.species_rule == "halves":
            ss.append((np.arange(n) >= n // 2).astype(np.uint8))
        else:
            raise ValueError(w.species_rule)
    f = _field(w)
    c0 = np.tile(f, w.n_inst)
    return {"x0": np.ascontiguousarray(np.concatenate(xs, 0)),
            "species0": np.ascontiguousarray(np.concatenate(ss, 0)),
            "c0": np.ascontiguousarray(c0)}
