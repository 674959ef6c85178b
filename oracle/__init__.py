"""FP64 CPU oracle of the hybrid chemotaxis step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``oracle.c`` (built with
gcc into ``liboracle.so`` next to it by :func:`build`) and shares no code
with the GPU library.

Function map (all arrays are numpy, float64 unless stated):

* :func:`philox`            Philox4x32-10 words for explicit counters / keys
* :func:`normals`           Box-Muller normals of one instance at one step
* :func:`forces`            pair repulsion at every agent (all-pairs or cell list)
* :func:`neighbours_f32`    float32-decided neighbour sets: counts and id hashes
* :func:`gradient`          node gradients of c
* :func:`interp`            multilinear interpolation of a node field
* :func:`drift`             chi * interpolated gradient at every agent
* :func:`deposit`           piecewise-linear deposit of source / uptake
* :func:`pde`               n_sub forward-Euler updates of the chemical
* :func:`pde_density`       the same updates from densities (kernel density deposit)
* :func:`deposit_kde`       Gaussian kernel density of source / uptake at the nodes
  (:func:`deposit_kde_at` at chosen nodes only)
* :func:`react`             type switching of one step (eq. Chemo_reactions)
* :func:`hs_correct`        hard-sphere overlap correction
* :func:`step` / :func:`run` whole time steps of one instance
* :func:`density_loss`      smoothed-histogram loss of the differentiation runs
* :func:`species_hist`, :func:`field_mean`  ensemble statistics

Pins (``tests/test_oracle_*.py``, all CPU): Philox against rocRAND's
philox4x32_10 engine compiled for the host; normals by
moments and KS; neighbour sets against a k-d tree and all-pairs search;
forces by two-agent closed forms and Newton's third law; interpolation,
gradient and deposit by exact affine cases, the deposit / interpolation
duality and mass; the PDE by its exact discrete Fourier decay and mass
invariants; free diffusion and constant drift by their MSD and mean laws;
type switching by the two-state Markov chain; the kernel density by its
mass, second moment and peak value; the potential variants by the force as
minus the energy gradient, pair closed forms and the hard-sphere invariants;
the ensemble statistics by brute-force counts.  The coupled
multi-step trajectory (``run`` over many steps) has no printed values in the
paper: beyond the per-step pins and the MSD / drift laws it is **parity
unpinned**.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB = _HERE / "liboracle.so"
MAX_SPECIES = 8


def build(force: bool = True) -> Path:
    """Compile oracle.c with gcc (FP64, OpenMP, no FMA contraction)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", str(_SRC), "-o", str(tmp), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("periodic", C.c_int32), ("L", C.c_double),
                ("grid_n", C.c_int32), ("n_sub", C.c_int32),
                ("dt", C.c_double), ("k", C.c_double), ("D_c", C.c_double),
                ("gamma", C.c_double), ("n_species", C.c_int32), ("mode", C.c_int32),
                ("diam", C.c_double * MAX_SPECIES), ("D", C.c_double * MAX_SPECIES),
                ("chi", C.c_double * MAX_SPECIES), ("source", C.c_double * MAX_SPECIES),
                ("uptake", C.c_double * MAX_SPECIES), ("react_to", C.c_int32 * MAX_SPECIES),
                ("react_rate", C.c_double * MAX_SPECIES),
                ("react_rate_c", C.c_double * MAX_SPECIES), ("seed", C.c_uint64),
                ("inst", C.c_uint32), ("chi_scale", C.c_double),
                ("deposit_kernel", C.c_int32), ("kde_radius", C.c_double),
                ("potential", C.c_int32), ("tamed", C.c_int32), ("pot_range", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build()
        L = C.CDLL(str(_LIB))
        P = C.POINTER(Params)
        vp = C.c_void_p
        i64 = C.c_int64
        sig = {
            "orc_num_threads": ([], C.c_int),
            "orc_set_threads": ([C.c_int], None),
            "orc_philox_batch": ([i64, vp, vp, vp], None),
            "orc_normals": ([P, C.c_uint32, i64, vp, vp], None),
            "orc_forces": ([P, i64, vp, vp, vp], None),
            "orc_forces_subset": ([P, i64, vp, vp, i64, vp, vp], None),
            "orc_neighbours_f32": ([C.c_int, C.c_int, C.c_float, i64, vp, vp, vp, vp, C.c_int,
                                    C.c_int, vp, vp], None),
            "orc_hash_id": ([C.c_uint32], C.c_uint64),
            "orc_gradient": ([P, vp, vp], None),
            "orc_interp": ([P, vp, i64, vp, vp], None),
            "orc_drift": ([P, vp, i64, vp, vp, vp], None),
            "orc_deposit": ([P, i64, vp, vp, vp, vp], None),
            "orc_pde": ([P, vp, vp, vp], None),
            "orc_pde_density": ([P, vp, vp, vp], None),
            "orc_deposit_kde": ([P, i64, vp, vp, vp, vp], None),
            "orc_deposit_kde_at": ([P, i64, vp, vp, i64, vp, vp, vp], None),
            "orc_hs_correct": ([P, i64, vp, vp], None),
            "orc_react": ([P, i64, vp, vp, vp, vp, C.c_uint32, vp], None),
            "orc_step": ([P, i64, vp, vp, vp, vp, vp], None),
            "orc_run": ([P, i64, vp, vp, vp, vp, vp, C.c_int], None),
            "orc_density_loss": ([C.c_int, C.c_double, i64, vp, C.c_int, C.c_double, vp, vp],
                                 C.c_double),
            "orc_density_hist": ([C.c_int, C.c_double, i64, vp, C.c_int, C.c_double, vp], None),
            "orc_species_hist": ([C.c_int, C.c_double, i64, vp, vp, C.c_int, C.c_int, vp, vp],
                                 None),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def auto_substeps(dim: int, periodic: bool, L: float, grid_n: int, dt: float, D_c: float) -> int:
    """Smallest substep count keeping D_c dt' / h^2 within 90% of the
    explicit limit 1/(2 dim) of forward Euler with the centred Laplacian."""
    h = L / grid_n if periodic else L / (grid_n - 1)
    r = D_c * dt / (h * h)
    return max(1, math.ceil(r / (0.9 / (2 * dim))))


def params(w, inst: int = 0, mode: int = 1, **over) -> Params:
    """Oracle parameters of instance `inst` of a workloads.Workload."""
    p = Params()
    p.dim = w.dim
    p.periodic = 1 if w.periodic else 0
    p.L = w.L
    p.grid_n = w.grid_n
    p.n_sub = w.pde_substeps or auto_substeps(w.dim, w.periodic, w.L, w.grid_n, w.dt, w.D_c)
    p.dt, p.k, p.D_c, p.gamma = w.dt, w.k, w.D_c, w.gamma
    p.n_species = len(w.species)
    for s in range(MAX_SPECIES):
        p.react_to[s] = -1
    for s, sp in enumerate(w.species):
        p.diam[s], p.D[s], p.chi[s] = sp.diameter, sp.D, sp.chi
        p.source[s], p.uptake[s] = sp.source, sp.uptake
        p.react_to[s] = getattr(sp, "react_to", -1)
        p.react_rate[s] = getattr(sp, "react_rate", 0.0)
        p.react_rate_c[s] = getattr(sp, "react_rate_c", 0.0)
    ins = w.instances[inst]
    p.seed = ins.seed & (2**64 - 1)
    p.inst = ins.stream if getattr(ins, "stream", -1) >= 0 else inst
    p.chi_scale = ins.chi_scale
    p.mode = mode
    p.deposit_kernel = getattr(w, "deposit_kernel", 0)
    p.kde_radius = getattr(w, "kde_radius", 3.0)
    p.potential = getattr(w, "potential", 0)
    p.tamed = 1 if getattr(w, "tamed", False) else 0
    p.pot_range = getattr(w, "pot_range", 3.0)
    for k, v in over.items():
        setattr(p, k, v)
    return p


def num_threads() -> int:
    return lib().orc_num_threads()


def set_threads(n: int) -> None:
    lib().orc_set_threads(n)


def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    ctr = _c(ctr, np.uint32).reshape(-1, 4)
    key = _c(key, np.uint32).reshape(-1, 2)
    out = np.empty_like(ctr)
    lib().orc_philox_batch(len(ctr), _ptr(ctr), _ptr(key), _ptr(out))
    return out


def normals(p: Params, step: int, ids: np.ndarray) -> np.ndarray:
    ids = _c(ids, np.uint32)
    out = np.empty((len(ids), p.dim), np.float64)
    lib().orc_normals(C.byref(p), step, len(ids), _ptr(ids), _ptr(out))
    return out


def forces(p: Params, X: np.ndarray, sp: np.ndarray) -> np.ndarray:
    X = _c(X, np.float64)
    sp = _c(sp, np.uint8)
    F = np.empty_like(X)
    lib().orc_forces(C.byref(p), len(X), _ptr(X), _ptr(sp), _ptr(F))
    return F


def forces_subset(p: Params, X: np.ndarray, sp: np.ndarray, which: np.ndarray) -> np.ndarray:
    X = _c(X, np.float64)
    sp = _c(sp, np.uint8)
    which = _c(which, np.int64)
    F = np.empty((len(which), p.dim), np.float64)
    lib().orc_forces_subset(C.byref(p), len(X), _ptr(X), _ptr(sp), len(which), _ptr(which),
                            _ptr(F))
    return F


def cut2_table(diameters) -> np.ndarray:
    """float32 squared contact distances ((d_a + d_b) / 2)^2, rounded once."""
    d = np.asarray(diameters, np.float64)
    m = 0.5 * (d[:, None] + d[None, :])
    return np.ascontiguousarray((m * m).astype(np.float32))


def neighbours_f32(dim: int, periodic: bool, L: float, X: np.ndarray, sp: np.ndarray,
                   ids: np.ndarray, diameters, mode: int = 1):
    X = _c(X, np.float32)
    sp = _c(sp, np.uint8)
    ids = _c(ids, np.uint32)
    cut2 = cut2_table(diameters)
    n = len(X)
    cnt = np.empty(n, np.uint32)
    h = np.empty(n, np.uint64)
    lib().orc_neighbours_f32(dim, 1 if periodic else 0, float(L), n, _ptr(X), _ptr(sp),
                             _ptr(ids), _ptr(cut2), cut2.shape[0], mode, _ptr(cnt), _ptr(h))
    return cnt, h


def hash_id(i: int) -> int:
    return int(lib().orc_hash_id(i))


def n_nodes(p: Params) -> int:
    return p.grid_n ** p.dim


def gradient(p: Params, c: np.ndarray) -> np.ndarray:
    c = _c(c, np.float64)
    g = np.empty(p.dim * n_nodes(p), np.float64)
    lib().orc_gradient(C.byref(p), _ptr(c), _ptr(g))
    return g.reshape(p.dim, -1)


def interp(p: Params, f: np.ndarray, X: np.ndarray) -> np.ndarray:
    f = _c(f, np.float64)
    X = _c(X, np.float64)
    out = np.empty(len(X), np.float64)
    lib().orc_interp(C.byref(p), _ptr(f), len(X), _ptr(X), _ptr(out))
    return out


def drift(p: Params, c: np.ndarray, X: np.ndarray, sp: np.ndarray) -> np.ndarray:
    c = _c(c, np.float64)
    X = _c(X, np.float64)
    sp = _c(sp, np.uint8)
    out = np.empty_like(X)
    lib().orc_drift(C.byref(p), _ptr(c), len(X), _ptr(X), _ptr(sp), _ptr(out))
    return out


def deposit(p: Params, X: np.ndarray, sp: np.ndarray):
    X = _c(X, np.float64)
    sp = _c(sp, np.uint8)
    Ss = np.empty(n_nodes(p), np.float64)
    Su = np.empty(n_nodes(p), np.float64)
    lib().orc_deposit(C.byref(p), len(X), _ptr(X), _ptr(sp), _ptr(Ss), _ptr(Su))
    return Ss, Su


def deposit_kde(p: Params, X: np.ndarray, sp: np.ndarray):
    """Gaussian kernel density of source and uptake at every node: (sigma, upsilon)."""
    X = _c(X, np.float64)
    sp = _c(sp, np.uint8)
    sig = np.empty(n_nodes(p), np.float64)
    ups = np.empty(n_nodes(p), np.float64)
    lib().orc_deposit_kde(C.byref(p), len(X), _ptr(X), _ptr(sp), _ptr(sig), _ptr(ups))
    return sig, ups


def deposit_kde_at(p: Params, X: np.ndarray, sp: np.ndarray, nodes: np.ndarray):
    """The kernel density of source and uptake at the given flat node indices
    only (same definition as :func:`deposit_kde`): (sigma, upsilon)."""
    X = _c(X, np.float64)
    sp = _c(sp, np.uint8)
    nodes = _c(nodes, np.int64)
    sig = np.empty(len(nodes), np.float64)
    ups = np.empty(len(nodes), np.float64)
    lib().orc_deposit_kde_at(C.byref(p), len(X), _ptr(X), _ptr(sp), len(nodes), _ptr(nodes),
                             _ptr(sig), _ptr(ups))
    return sig, ups


def hs_correct(p: Params, X: np.ndarray, sp: np.ndarray) -> np.ndarray:
    """Hard-sphere overlap correction of positions X (returns a new array)."""
    X = _c(X, np.float64).copy()
    lib().orc_hs_correct(C.byref(p), len(X), _ptr(X), _ptr(_c(sp, np.uint8)))
    return X


def pde_density(p: Params, c: np.ndarray, sigma: np.ndarray, ups: np.ndarray) -> np.ndarray:
    c = _c(c, np.float64).copy()
    lib().orc_pde_density(C.byref(p), _ptr(c), _ptr(_c(sigma, np.float64)),
                          _ptr(_c(ups, np.float64)))
    return c


def pde(p: Params, c: np.ndarray, S_src: np.ndarray, S_upt: np.ndarray) -> np.ndarray:
    c = _c(c, np.float64).copy()
    S_src = _c(S_src, np.float64)
    S_upt = _c(S_upt, np.float64)
    lib().orc_pde(C.byref(p), _ptr(c), _ptr(S_src), _ptr(S_upt))
    return c


def run(p: Params, X: np.ndarray, sp: np.ndarray, c: np.ndarray, step: int, n_steps: int,
        ids: np.ndarray | None = None, return_species: bool = False):
    """Advance one instance by n_steps; returns (X, c, step[, species]) as new arrays."""
    X = _c(X, np.float64).copy()
    c = _c(c, np.float64).copy()
    sp = _c(sp, np.uint8).copy()
    ids = np.arange(len(X), dtype=np.uint32) if ids is None else _c(ids, np.uint32)
    st = C.c_uint32(step)
    lib().orc_run(C.byref(p), len(X), _ptr(X), _ptr(sp), _ptr(ids), _ptr(c), C.byref(st), n_steps)
    return (X, c, st.value, sp) if return_species else (X, c, st.value)


def step(p: Params, X, sp, c, step_no: int, ids=None, return_species: bool = False):
    return run(p, X, sp, c, step_no, 1, ids, return_species)


def react(p: Params, X: np.ndarray, sp: np.ndarray, c: np.ndarray, step_no: int,
          ids: np.ndarray | None = None) -> np.ndarray:
    """Species after the type-switching draw of step `step_no` (eq. Chemo_reactions)."""
    X = _c(X, np.float64)
    sp = _c(sp, np.uint8)
    c = _c(c, np.float64)
    ids = np.arange(len(X), dtype=np.uint32) if ids is None else _c(ids, np.uint32)
    out = np.empty(len(X), np.uint8)
    lib().orc_react(C.byref(p), len(X), _ptr(X), _ptr(sp), _ptr(ids), _ptr(c), step_no, _ptr(out))
    return out


def density_loss(dim: int, L: float, X: np.ndarray, target: np.ndarray, hist_n: int = 64,
                 sigma_bins: float = 2.0, grad: bool = False):
    """Smoothed-histogram mismatch of one instance's positions (FP64)."""
    X = _c(X, np.float64)
    target = _c(target, np.float64)
    g = np.empty_like(X) if grad else None
    loss = lib().orc_density_loss(dim, L, len(X), _ptr(X), hist_n, sigma_bins, _ptr(target),
                                  _ptr(g) if grad else None)
    return (loss, g) if grad else loss


def density_hist(dim: int, L: float, X: np.ndarray, hist_n: int = 64, sigma_bins: float = 2.0):
    X = _c(X, np.float64)
    out = np.empty(hist_n ** dim, np.float64)
    lib().orc_density_hist(dim, L, len(X), _ptr(X), hist_n, sigma_bins, _ptr(out))
    return out


def target_hist(w, inputs: dict, n_steps: int, hist_n: int = 64, sigma_bins: float = 2.0):
    """Smoothed histograms (all instances) after an oracle run of a workload."""
    X, _ = run_workload(w, inputs, n_steps)
    out, off = [], 0
    for ins in w.instances:
        out.append(density_hist(w.dim, w.L, X[off:off + ins.n_agents], hist_n, sigma_bins))
        off += ins.n_agents
    return np.concatenate(out)


def workload_at(w, theta):
    """The workload with chi of the chemotactic species, k and every
    species' D replaced by theta = (chi, k, D)."""
    import dataclasses
    chi, k, D = (float(v) for v in theta)
    sp = tuple(dataclasses.replace(s, D=D, chi=chi if s.chi != 0.0 else 0.0) for s in w.species)
    return dataclasses.replace(w, species=sp, k=k)


def loss_at(w, inputs: dict, theta, target: np.ndarray, n_steps: int, hist_n: int = 64,
            sigma_bins: float = 2.0) -> float:
    """FP64 loss after n_steps from `inputs` at theta (summed over instances)."""
    wt = workload_at(w, theta)
    X, _ = run_workload(wt, inputs, n_steps)
    H = hist_n ** w.dim
    tot, off = 0.0, 0
    for k, ins in enumerate(w.instances):
        n = ins.n_agents
        tot += density_loss(w.dim, w.L, X[off:off + n], target[k * H:(k + 1) * H], hist_n,
                            sigma_bins)
        off += n
    return tot


def run_workload(w, inputs: dict, n_steps: int, mode: int = 1, step0: int = 0,
                 return_species: bool = False):
    """Advance every instance of a workload from `inputs` (workloads.make_inputs)."""
    xs, cs, ss = [], [], []
    off = 0
    G = w.grid_n ** w.dim
    for k, ins in enumerate(w.instances):
        n = ins.n_agents
        p = params(w, k, mode=mode)
        X, c, _, s = run(p, inputs["x0"][off:off + n], inputs["species0"][off:off + n],
                         inputs["c0"][k * G:(k + 1) * G], step0, n_steps, return_species=True)
        xs.append(X)
        cs.append(c)
        ss.append(s)
        off += n
    out = (np.concatenate(xs, 0), np.concatenate(cs, 0))
    return out + (np.concatenate(ss, 0),) if return_species else out


def species_hist(dim: int, L: float, X: np.ndarray, sp: np.ndarray, n_species: int, hist_n: int):
    """Per-species position histograms over all realisations (float32 positions)
    and the species totals: (counts[n_species, hist_n^dim], totals[n_species])."""
    X = _c(X, np.float32)
    sp = _c(sp, np.uint8)
    counts = np.empty(n_species * hist_n ** dim, np.uint32)
    totals = np.empty(n_species, np.uint32)
    lib().orc_species_hist(dim, L, len(sp), _ptr(X), _ptr(sp), n_species, hist_n, _ptr(counts),
                           _ptr(totals))
    return counts.reshape(n_species, -1), totals


def field_mean(c: np.ndarray, n_inst: int) -> np.ndarray:
    """Mean of the chemical over realisations, node by node (FP64)."""
    return np.asarray(c, np.float64).reshape(n_inst, -1).mean(0)
