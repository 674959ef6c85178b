"""The C ABI library (CPU side only): it loads, exports every entry point
that include/pc.h declares, and its host-only calls validate parameters."""
import ctypes as C
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "pc.h"


def _declared():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pc_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    from paper_1805_11007_amd import _lib
    assert set(_declared()) == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_1805_11007_amd import _lib
    if not _lib.LIB_PATH.exists():
        pytest.skip("libpc.so not built")
    lib = C.CDLL(str(_lib.LIB_PATH))
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def _spec(**over):
    from paper_1805_11007_amd import InstanceSpec, ModelSpec, SpeciesSpec
    kw = dict(dim=2, periodic=True, L=1.0, grid_n=64, dt=1e-5, k=100.0, D_c=1.0, gamma=0.1,
              species=[SpeciesSpec(0.01, 1.0, 1.0, 1.0, 0.0)],
              instances=[InstanceSpec(1000, 1)])
    kw.update(over)
    return ModelSpec(**kw)


def test_workspace_bytes_and_validation():
    from paper_1805_11007_amd import InstanceSpec, PcError, SpeciesSpec, workspace_bytes
    from paper_1805_11007_amd import _lib
    if not _lib.LIB_PATH.exists():
        pytest.skip("libpc.so not built")
    n1 = workspace_bytes(_spec())
    n2 = workspace_bytes(_spec(instances=[InstanceSpec(1000, 1)] * 3))
    assert 0 < n1 < n2
    assert workspace_bytes(_spec(), adjoint_steps=10) > n1
    bad = [dict(dim=4), dict(grid_n=2), dict(species=[SpeciesSpec(0.0, 1.0)]),
           dict(species=[SpeciesSpec(0.6, 1.0)]), dict(instances=[InstanceSpec(0, 1)]),
           dict(pde_substeps=1, dt=1e-2), dict(bin_size=0.001), dict(block=100)]
    for over in bad:
        with pytest.raises(PcError):
            workspace_bytes(_spec(**over))
    L = _lib.load()
    assert L.pc_strerror(-2).decode().startswith("explicit PDE")


def test_validation_of_variant_parameters():
    """Host-side checks of the switching, deposit and potential options."""
    from paper_1805_11007_amd import PcError, SpeciesSpec, workspace_bytes
    from paper_1805_11007_amd import _lib
    if not _lib.LIB_PATH.exists():
        pytest.skip("libpc.so not built")
    two = [SpeciesSpec(0.01, 1.0), SpeciesSpec(0.01, 1.0)]
    ok = [dict(species=[SpeciesSpec(0.01, 1.0, react_to=1, react_rate=5.0), two[1]]),
          dict(species=[SpeciesSpec(0.01, 1.0, react_to=0, react_rate=0.0)]),  # no rate: no switch
          dict(deposit_kernel=1, kde_radius=4.0), dict(potential=1, pot_range=2.0),
          dict(potential=2), dict(tamed=True), dict(deposit_mode=2), dict(deposit_mode=4),
          dict(deposit_mode=4, slab_split=1)]
    for over in ok:
        assert workspace_bytes(_spec(**over)) > 0, over
    bad = [dict(species=[SpeciesSpec(0.01, 1.0, react_to=2, react_rate=5.0), two[1]]),
           dict(species=[SpeciesSpec(0.01, 1.0, react_to=0, react_rate=5.0)]),   # to itself
           dict(species=[SpeciesSpec(0.01, 1.0, react_to=1, react_rate=-1.0), two[1]]),
           dict(species=[SpeciesSpec(0.01, 1.0, react_to=1, react_rate_c=float("inf")), two[1]]),
           dict(deposit_kernel=2), dict(deposit_kernel=1, kde_radius=60.0),
           dict(deposit_kernel=1, deposit_mode=3), dict(deposit_kernel=1, potential=2),
           dict(potential=3), dict(potential=1, pot_range=0.5), dict(potential=1, pot_range=60.0),
           dict(deposit_kernel=1, deposit_mode=4), dict(deposit_mode=5),
           dict(deposit_mode=4, slab_split=-1)]
    for over in bad:
        with pytest.raises(PcError):
            workspace_bytes(_spec(**over))


def test_create_reports_enospace_and_bad_workspace_before_any_device_work():
    """pc_create validates the workspace on the host before it enqueues
    anything: a workspace one byte short gives PC_ENOSPACE, a misaligned one
    PC_EINVAL.  The device pointers are never dereferenced on these paths
    (placeholders are passed), so no GPU is needed."""
    import ctypes as C
    from paper_1805_11007_amd import _lib
    from paper_1805_11007_amd._lib import PC_EINVAL, PC_ENOSPACE
    if not _lib.LIB_PATH.exists():
        pytest.skip("libpc.so not built")
    L = _lib.load()
    cfg, sp, ns, inst, ni = _spec().c_structs()
    need = L.pc_workspace_bytes(C.byref(cfg), sp, ns, inst, ni)
    assert need > 0
    out = C.c_void_p()
    fake = C.c_void_p(1 << 20)      # 256-byte aligned placeholder, never touched
    rc = L.pc_create(C.byref(cfg), sp, ns, inst, ni, fake, need - 1, fake, fake, fake, None,
                     C.byref(out))
    assert rc == PC_ENOSPACE and not out.value
    assert b"workspace too small" in L.pc_last_error()
    rc = L.pc_create(C.byref(cfg), sp, ns, inst, ni, C.c_void_p((1 << 20) + 16), need, fake,
                     fake, fake, None, C.byref(out))
    assert rc == PC_EINVAL and not out.value
    rc = L.pc_create(C.byref(cfg), sp, ns, inst, ni, fake, need, None, fake, fake, None,
                     C.byref(out))
    assert rc == PC_EINVAL and not out.value
