"""MI355X (gfx950) implementation of the per-step hot path of the hybrid
chemotaxis model of Bruna, Maini & Robinson (arXiv:1805.11007).

The computation lives in ``libpc.so`` (HIP kernels behind the C ABI of
``include/pc.h``); this package is its thin Python binding plus host-side
helpers (autotuner, differentiable run).
"""
from ._lib import PcError, load  # noqa: F401
from .sim import InstanceSpec, ModelSpec, Sim, SpeciesSpec, workspace_bytes  # noqa: F401

__all__ = ["Sim", "ModelSpec", "SpeciesSpec", "InstanceSpec", "PcError", "load",
           "workspace_bytes"]
