"""PyTorch-facing wrapper of the C ABI: device memory and streams come from
torch, all computation from the library's kernels.

The object mirrors the paper's ``Simulation`` class (Sect. 4): construct it
with a model description and an initial state, ``integrate(T)`` or
``step(n)`` it, and read ``positions()``, ``species()`` (the paper's
``get_type``) and ``field()`` back as torch tensors on the GPU.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Sequence

import torch

from . import _lib as LB


@dataclass
class SpeciesSpec:
    diameter: float
    D: float
    chi: float = 0.0
    source: float = 0.0
    uptake: float = 0.0
    react_to: int = -1        # species switched to (eq. Chemo_reactions); -1: none
    react_rate: float = 0.0   # switching rate react_rate + react_rate_c * c(X)
    react_rate_c: float = 0.0


@dataclass
class InstanceSpec:
    n_agents: int
    seed: int
    chi_scale: float = 1.0
    stream: int = -1     # noise stream index; -1: position in the instance list


@dataclass
class ModelSpec:
    dim: int
    periodic: bool
    L: float
    grid_n: int
    dt: float
    k: float
    D_c: float
    gamma: float
    species: Sequence[SpeciesSpec]
    instances: Sequence[InstanceSpec]
    pde_substeps: int = 0
    bin_size: float = 0.0
    deterministic: bool = False
    block: int = 0
    deposit_mode: int = 0    # 0 auto, 1 LDS-aggregated, 2 direct atomics, 3 fused per instance,
                             # 4 owner-computes node slabs (3D)
    deposit_kernel: int = 0  # 0 particle-in-cell, 1 Gaussian kernel density (Sect. 2.3)
    slab_split: int = 0      # slab deposit: agents above which a slab is handed over (0: 2048)
    kde_radius: float = 0.0  # kernel truncation in bandwidths (0: 3)
    potential: int = 0       # 0 harmonic, 1 exponential k exp(-r/d), 2 hard spheres
    tamed: bool = False      # tamed Euler pair drift (eq. sde_ETamed)
    pot_range: float = 0.0   # exponential range in contact distances (0: 3)

    @classmethod
    def from_workload(cls, w, **over) -> "ModelSpec":
        """Build from any object with the attributes of a workload description."""
        sp = [SpeciesSpec(s.diameter, s.D, s.chi, s.source, s.uptake,
                          getattr(s, "react_to", -1), getattr(s, "react_rate", 0.0),
                          getattr(s, "react_rate_c", 0.0)) for s in w.species]
        ins = [InstanceSpec(i.n_agents, i.seed, i.chi_scale, getattr(i, 'stream', -1))
               for i in w.instances]
        kw = dict(dim=w.dim, periodic=w.periodic, L=w.L, grid_n=w.grid_n, dt=w.dt, k=w.k,
                  D_c=w.D_c, gamma=w.gamma, species=sp, instances=ins,
                  pde_substeps=w.pde_substeps, deposit_kernel=getattr(w, "deposit_kernel", 0),
                  kde_radius=getattr(w, "kde_radius", 0.0),
                  potential=getattr(w, "potential", 0), tamed=bool(getattr(w, "tamed", False)),
                  pot_range=getattr(w, "pot_range", 0.0))
        kw.update(over)
        return cls(**kw)

    def c_structs(self):
        cfg = LB.PcConfig()
        cfg.dim = self.dim
        cfg.periodic = 1 if self.periodic else 0
        cfg.L = self.L
        cfg.grid_n = self.grid_n
        cfg.dt = self.dt
        cfg.k_rep = self.k
        cfg.D_c = self.D_c
        cfg.gamma = self.gamma
        cfg.pde_substeps = self.pde_substeps
        cfg.bin_size = self.bin_size
        cfg.deterministic = 1 if self.deterministic else 0
        cfg.block = self.block
        cfg.bin_order = 0
        cfg.deposit_mode = self.deposit_mode
        cfg.deposit_kernel = self.deposit_kernel
        cfg.slab_split = self.slab_split
        cfg.kde_radius = self.kde_radius
        cfg.potential = self.potential
        cfg.tamed = 1 if self.tamed else 0
        cfg.pot_range = self.pot_range
        ns = len(self.species)
        sp = (LB.PcSpecies * max(ns, 1))()
        for k, s in enumerate(self.species):
            sp[k].diameter, sp[k].D, sp[k].chi = s.diameter, s.D, s.chi
            sp[k].source, sp[k].uptake = s.source, s.uptake
            sp[k].react_to = int(s.react_to)
            sp[k].react_rate, sp[k].react_rate_c = float(s.react_rate), float(s.react_rate_c)
        ni = len(self.instances)
        ins = (LB.PcInstance * max(ni, 1))()
        for k, i in enumerate(self.instances):
            ins[k].n_agents = int(i.n_agents)
            ins[k].seed = int(i.seed) & (2**64 - 1)
            ins[k].chi_scale = float(i.chi_scale)
            ins[k].stream = int(getattr(i, "stream", -1))
        return cfg, sp, ns, ins, ni

    @property
    def n_total(self) -> int:
        return sum(int(i.n_agents) for i in self.instances)

    @property
    def n_nodes(self) -> int:
        return len(self.instances) * self.grid_n ** self.dim


def _ptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def workspace_bytes(spec: ModelSpec, adjoint_steps: int = 0) -> int:
    L = LB.load()
    cfg, sp, ns, ins, ni = spec.c_structs()
    if adjoint_steps > 0:
        n = L.pc_workspace_bytes_adjoint(C.byref(cfg), sp, ns, ins, ni, adjoint_steps)
    else:
        n = L.pc_workspace_bytes(C.byref(cfg), sp, ns, ins, ni)
    if n == 0:
        raise LB.PcError(LB.PC_EINVAL, "invalid parameters: " + L.pc_last_error().decode())
    return int(n)


class Sim:
    """One handle of the library: a model plus n_inst instances on one GPU."""

    def __init__(self, spec: ModelSpec, x0: torch.Tensor, species0: torch.Tensor,
                 c0: torch.Tensor, device: str | torch.device = "cuda",
                 stream: torch.cuda.Stream | None = None, adjoint_steps: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the chemotaxis library needs a ROCm GPU")
        self.L = LB.load()
        self.spec = spec
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream or torch.cuda.current_stream(self.device)
        self._cfg = spec.c_structs()
        nbytes = workspace_bytes(spec, adjoint_steps)
        # torch's allocator returns blocks aligned to at least 512 bytes
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        n, d = spec.n_total, spec.dim
        x0 = x0.to(self.device, torch.float32).contiguous().reshape(n, d)
        species0 = species0.to(self.device, torch.uint8).contiguous().reshape(n)
        c0 = c0.to(self.device, torch.float32).contiguous().reshape(spec.n_nodes)
        cfg, sp, ns, ins, ni = self._cfg
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            LB.check(self.L.pc_create(C.byref(cfg), sp, ns, ins, ni, _ptr(self.workspace),
                                      nbytes, _ptr(x0), _ptr(species0), _ptr(c0),
                                      C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        info = LB.PcInfo()
        LB.check(self.L.pc_info(self.h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in LB.PcInfo._fields_}

    # -- stepping ---------------------------------------------------------
    def step(self, n: int = 1) -> None:
        LB.check(self.L.pc_step(self.h, int(n)))

    def integrate(self, T: float) -> None:
        """Advance by time T: round(T / dt) steps."""
        self.step(int(round(T / self.spec.dt)))

    def use_graph(self, on: bool = True) -> None:
        LB.check(self.L.pc_use_graph(self.h, 1 if on else 0))

    # -- outputs ----------------------------------------------------------
    def positions(self, out: torch.Tensor | None = None) -> torch.Tensor:
        out = out if out is not None else torch.empty(self.spec.n_total, self.spec.dim,
                                                      dtype=torch.float32, device=self.device)
        LB.check(self.L.pc_positions(self.h, _ptr(out)))
        return out

    def field(self, out: torch.Tensor | None = None) -> torch.Tensor:
        out = out if out is not None else torch.empty(self.spec.n_nodes, dtype=torch.float32,
                                                      device=self.device)
        LB.check(self.L.pc_field(self.h, _ptr(out)))
        return out

    def species(self) -> torch.Tensor:
        out = torch.empty(self.spec.n_total, dtype=torch.uint8, device=self.device)
        LB.check(self.L.pc_species(self.h, _ptr(out)))
        return out

    get_positions = positions
    get_type = species

    def get_state(self):
        x = torch.empty(self.spec.n_total, self.spec.dim, dtype=torch.float32, device=self.device)
        c = torch.empty(self.spec.n_nodes, dtype=torch.float32, device=self.device)
        st = C.c_uint32()
        LB.check(self.L.pc_get_state(self.h, _ptr(x), _ptr(c), C.byref(st)))
        return x, c, int(st.value)

    def set_state(self, x: torch.Tensor, c: torch.Tensor, step: int) -> None:
        x = x.to(self.device, torch.float32).contiguous()
        c = c.to(self.device, torch.float32).contiguous()
        LB.check(self.L.pc_set_state(self.h, _ptr(x), _ptr(c), int(step)))
        self._keep = (x, c)  # inputs must live until the stream has read them

    def set_species(self, species: torch.Tensor) -> None:
        """Species of every agent (id order); also what set_state restores."""
        species = species.to(self.device, torch.uint8).contiguous().reshape(self.spec.n_total)
        LB.check(self.L.pc_set_species(self.h, _ptr(species)))
        self._keep_sp = species  # must live until the stream has read it

    def ensemble_stats(self, hist_n: int, field_mean: bool = True):
        """Per-species histograms summed over instances (n_species x
        hist_n^dim, int32 view of uint32 counts), species totals and the
        instance-mean field (None if not asked for)."""
        ns = len(self.spec.species)
        counts = torch.empty(ns * hist_n ** self.spec.dim, dtype=torch.int32, device=self.device)
        totals = torch.empty(ns, dtype=torch.int32, device=self.device)
        cm = torch.empty(self.spec.grid_n ** self.spec.dim, dtype=torch.float32,
                         device=self.device) if field_mean else None
        LB.check(self.L.pc_ensemble_stats(self.h, int(hist_n), _ptr(counts), _ptr(totals),
                                          _ptr(cm) if field_mean else C.c_void_p(0)))
        return counts.view(ns, -1), totals, cm

    def sync(self) -> None:
        LB.check(self.L.pc_sync(self.h))

    def warnings(self) -> int:
        b = C.c_uint32()
        LB.check(self.L.pc_warnings(self.h, C.byref(b)))
        return int(b.value)

    def profile_steps(self, n: int) -> dict:
        """Run n steps with HIP events between stages; mean ms per stage."""
        out = (C.c_double * len(LB.STAGES))()
        LB.check(self.L.pc_profile_steps(self.h, int(n), out))
        return dict(zip(LB.STAGES, list(out)))

    # -- reverse mode ---------------------------------------------------------
    def adjoint_segment(self, lamX: torch.Tensor, lamC: torch.Tensor, n: int):
        """Reverse sweep over n steps from the current state (see pc.h).

        Returns (dL/dX, dL/dc) of the current state and an (n_inst, 3) array
        of derivatives with respect to scales of chi, k and D."""
        import numpy as np
        lamX = lamX.to(self.device, torch.float32).contiguous()
        lamC = lamC.to(self.device, torch.float32).contiguous()
        ox = torch.empty_like(lamX)
        oc = torch.empty_like(lamC)
        ni = len(self.spec.instances)
        dth = (C.c_double * (3 * ni))()
        LB.check(self.L.pc_adjoint_segment(self.h, _ptr(lamX), _ptr(lamC), int(n), _ptr(ox),
                                           _ptr(oc), dth))
        return ox, oc, np.array(list(dth), dtype=np.float64).reshape(ni, 3)

    def density_loss(self, target: torch.Tensor, hist_n: int = 64, sigma_bins: float = 2.0,
                     grad: bool = True):
        """Smoothed-histogram loss of the current positions per instance, and
        optionally its gradient with respect to the positions (id order)."""
        import numpy as np
        target = target.to(self.device, torch.float32).contiguous()
        nb = int(self.L.pc_density_loss_work_bytes(self.h, int(hist_n)))
        if nb == 0:
            raise LB.PcError(LB.PC_EINVAL, "bad histogram size")
        work = torch.empty(nb, dtype=torch.uint8, device=self.device)
        ni = len(self.spec.instances)
        loss = (C.c_double * ni)()
        g = torch.empty(self.spec.n_total, self.spec.dim, dtype=torch.float32,
                        device=self.device) if grad else None
        LB.check(self.L.pc_density_loss(self.h, _ptr(target), int(hist_n), float(sigma_bins),
                                        _ptr(work), nb, loss,
                                        _ptr(g) if grad else C.c_void_p(0)))
        return np.array(list(loss)), g

    def density_loss_noalloc(self, target: torch.Tensor, hist_n: int = 64,
                             sigma_bins: float = 2.0, dLdX: torch.Tensor | None = None):
        """density_loss through pc_density_loss_noalloc: the library uses its
        static scratch, so nothing is allocated for the call (target and the
        optional dL/dX output must already be float32 device tensors)."""
        import numpy as np
        if (target.dtype != torch.float32 or target.device != self.device
                or not target.is_contiguous()):
            raise ValueError("target must be a contiguous float32 tensor on the handle's device")
        if dLdX is not None and (dLdX.dtype != torch.float32 or dLdX.device != self.device
                                 or not dLdX.is_contiguous()):
            raise ValueError("dLdX must be a contiguous float32 tensor on the handle's device")
        ni = len(self.spec.instances)
        loss = (C.c_double * ni)()
        LB.check(self.L.pc_density_loss_noalloc(self.h, _ptr(target), int(hist_n),
                                                float(sigma_bins), loss,
                                                _ptr(dLdX) if dLdX is not None
                                                else C.c_void_p(0)))
        return np.array(list(loss))

    def density_hist(self, hist_n: int = 64, sigma_bins: float = 2.0) -> torch.Tensor:
        """Smoothed position histogram of the loss (n_inst x hist_n^dim)."""
        nb = int(self.L.pc_density_loss_work_bytes(self.h, int(hist_n)))
        if nb == 0:
            raise LB.PcError(LB.PC_EINVAL, "bad histogram size")
        work = torch.empty(nb, dtype=torch.uint8, device=self.device)
        out = torch.empty(len(self.spec.instances) * hist_n ** self.spec.dim,
                          dtype=torch.float32, device=self.device)
        LB.check(self.L.pc_density_hist(self.h, int(hist_n), float(sigma_bins), _ptr(work), nb,
                                        _ptr(out)))
        return out

    # -- debug --------------------------------------------------------------
    def debug_neighbours(self):
        cnt = torch.empty(self.spec.n_total, dtype=torch.int32, device=self.device)
        hsh = torch.empty(self.spec.n_total, dtype=torch.int64, device=self.device)
        LB.check(self.L.pc_debug_neighbours(self.h, _ptr(cnt), _ptr(hsh)))
        return cnt, hsh

    def debug_forces(self) -> torch.Tensor:
        F = torch.empty(self.spec.n_total, self.spec.dim, dtype=torch.float32, device=self.device)
        LB.check(self.L.pc_debug_forces(self.h, _ptr(F)))
        return F

    def close(self) -> None:
        if getattr(self, "h", None):
            self.L.pc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
