"""ctypes binding of libpc.so (the C ABI declared in include/pc.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libpc.so"

PC_OK, PC_EINVAL, PC_EUNSTABLE, PC_ENOSPACE, PC_EHIP, PC_ENONFINITE, PC_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
PC_WARN_DT_RULE, PC_WARN_POSITIVITY, PC_WARN_CLAMPED, PC_WARN_REACTION = 1, 2, 4, 8
MAX_SPECIES = 8

EXPORTS = (
    "pc_workspace_bytes", "pc_workspace_bytes_adjoint", "pc_create", "pc_step", "pc_use_graph",
    "pc_positions", "pc_field", "pc_species", "pc_get_state", "pc_set_state", "pc_set_species", "pc_ensemble_stats", "pc_sync",
    "pc_warnings", "pc_info", "pc_destroy", "pc_strerror", "pc_last_error",
    "pc_debug_neighbours", "pc_debug_forces", "pc_adjoint_segment", "pc_profile_steps",
    "pc_density_loss_work_bytes", "pc_density_loss", "pc_density_loss_noalloc", "pc_density_hist",
)
STAGES = ("bin", "scan", "scatter", "stable", "update", "deposit", "pde", "overlap")


class PcConfig(C.Structure):
    _fields_ = [("dim", C.c_int32), ("periodic", C.c_int32), ("L", C.c_double),
                ("grid_n", C.c_int32), ("dt", C.c_double), ("k_rep", C.c_double),
                ("D_c", C.c_double), ("gamma", C.c_double), ("pde_substeps", C.c_int32),
                ("bin_size", C.c_double), ("deterministic", C.c_int32), ("block", C.c_int32),
                ("bin_order", C.c_int32), ("deposit_mode", C.c_int32),
                ("deposit_kernel", C.c_int32), ("slab_split", C.c_int32),
                ("kde_radius", C.c_double), ("potential", C.c_int32), ("tamed", C.c_int32),
                ("pot_range", C.c_double)]


class PcSpecies(C.Structure):
    _fields_ = [("diameter", C.c_double), ("D", C.c_double), ("chi", C.c_double),
                ("source", C.c_double), ("uptake", C.c_double), ("react_to", C.c_int32),
                ("reserved", C.c_int32), ("react_rate", C.c_double), ("react_rate_c", C.c_double)]


class PcInstance(C.Structure):
    _fields_ = [("n_agents", C.c_int32), ("stream", C.c_int32), ("seed", C.c_uint64),
                ("chi_scale", C.c_double)]


class PcInfo(C.Structure):
    _fields_ = [("n_total", C.c_int32), ("n_inst", C.c_int32), ("bins_per_axis", C.c_int32),
                ("stencil", C.c_int32), ("n_bins_total", C.c_int64),
                ("n_nodes_total", C.c_int64), ("pde_substeps", C.c_int32),
                ("block", C.c_int32), ("bin_side", C.c_double), ("workspace_bytes", C.c_size_t),
                ("deposit_path", C.c_int32), ("reserved", C.c_int32)]


class PcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def load() -> C.CDLL:
    """Load libpc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1805_11007_amd.build` (or __graft_entry__.build())")
    L = C.CDLL(str(LIB_PATH))
    vp, i32, u32p = C.c_void_p, C.c_int, C.POINTER(C.c_uint32)
    cfgp, spp, inp = C.POINTER(PcConfig), C.POINTER(PcSpecies), C.POINTER(PcInstance)
    sigs = {
        "pc_workspace_bytes": ([cfgp, spp, i32, inp, i32], C.c_size_t),
        "pc_workspace_bytes_adjoint": ([cfgp, spp, i32, inp, i32, i32], C.c_size_t),
        "pc_create": ([cfgp, spp, i32, inp, i32, vp, C.c_size_t, vp, vp, vp, vp,
                       C.POINTER(vp)], i32),
        "pc_step": ([vp, i32], i32),
        "pc_use_graph": ([vp, i32], i32),
        "pc_positions": ([vp, vp], i32),
        "pc_field": ([vp, vp], i32),
        "pc_species": ([vp, vp], i32),
        "pc_get_state": ([vp, vp, vp, u32p], i32),
        "pc_set_state": ([vp, vp, vp, C.c_uint32], i32),
        "pc_set_species": ([vp, vp], i32),
        "pc_ensemble_stats": ([vp, i32, vp, vp, vp], i32),
        "pc_sync": ([vp], i32),
        "pc_warnings": ([vp, u32p], i32),
        "pc_info": ([vp, C.POINTER(PcInfo)], i32),
        "pc_destroy": ([vp], i32),
        "pc_strerror": ([i32], C.c_char_p),
        "pc_last_error": ([], C.c_char_p),
        "pc_debug_neighbours": ([vp, vp, vp], i32),
        "pc_debug_forces": ([vp, vp], i32),
        "pc_adjoint_segment": ([vp, vp, vp, i32, vp, vp, C.POINTER(C.c_double)], i32),
        "pc_profile_steps": ([vp, i32, C.POINTER(C.c_double)], i32),
        "pc_density_loss_work_bytes": ([vp, i32], C.c_size_t),
        "pc_density_loss": ([vp, vp, i32, C.c_double, vp, C.c_size_t, C.POINTER(C.c_double),
                             vp], i32),
        "pc_density_loss_noalloc": ([vp, vp, i32, C.c_double, C.POINTER(C.c_double), vp], i32),
        "pc_density_hist": ([vp, i32, C.c_double, vp, C.c_size_t, vp], i32),
    }
    for name, (args, res) in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != PC_OK:
        L = load()
        raise PcError(rc, f"{L.pc_strerror(rc).decode()}: {L.pc_last_error().decode()}")
