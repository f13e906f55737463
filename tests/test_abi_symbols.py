"""CPU check of the C-ABI library: it loads and exports every function declared in
include/mpm_gimp.h (no compute call is made without a GPU)."""
import ctypes as C
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "mpm_gimp.h"


def declared_functions():
    txt = HEADER.read_text()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int32_t|int64_t|void)\s+(\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("octree_build", "mpm_assemble", "mpm_assemble_adjoint", "mpm_mesh_info", "mpm_mesh_arrays",
              "mpm_mesh_free", "mpm_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_2606_09275_amd import _lib
    if not _lib.LIB_PATH.exists():
        from paper_2606_09275_amd.build import build
        build()
    L = C.CDLL(str(_lib.LIB_PATH))
    for name in declared_functions():
        assert hasattr(L, name), name
    assert sorted(_lib.EXPORTED) == declared_functions()


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2606_09275_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", tmp_path / "absent.so")
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()


def test_argument_checks_need_no_gpu():
    """Argument checks of the C ABI run before any device call: bad refinement criteria,
    null handles and bad GIMP-split arguments are refused with MPM_EARG (or MPM_ESTENCIL for
    a lattice beyond the key width) on a machine without a GPU."""
    from paper_2606_09275_amd import _lib
    from paper_2606_09275_amd.mesh import refine_struct
    if not _lib.LIB_PATH.exists():
        from paper_2606_09275_amd.build import build
        build()
    L = _lib.lib()
    base = dict(lo=(0.0, 0.0, 0.0), base=(2, 2, 2), h0=0.5, lvl_base=1, lvl_max=3, body_kind=0, body=(),
                dx_region=0.0)
    bad = [dict(base, lvl_max=0), dict(base, h0=0.0), dict(base, h0=float("nan")), dict(base, base=(0, 2, 2)),
           dict(base, body_kind=7), dict(base, dx_region=-1.0), dict(base, lvl_max=1 + 14)]
    h = C.c_void_p()
    for crit in bad:
        r = refine_struct(crit)
        assert L.octree_build(C.byref(r), None, None, 0, None, C.byref(h)) == _lib.MPM_EARG, crit
        assert not h.value
    r = refine_struct(dict(base, base=(4096, 2, 2), lvl_max=3))
    assert L.octree_build(C.byref(r), None, None, 0, None, C.byref(h)) == -3
    assert L.octree_build(None, None, None, 0, None, C.byref(h)) == _lib.MPM_EARG
    cnt = C.c_int64(0)
    assert L.mpm_split_mark(None, None, None, 0, C.c_double(2.0), None, C.byref(cnt), None) == _lib.MPM_EARG
    it, rr = C.c_int32(0), C.c_double(0.0)
    assert L.mpm_solve_gmres(None, 0, None, None, None, None, 1e-8, 30, 100, C.byref(it), C.byref(rr),
                             None) == _lib.MPM_EARG
    info = _lib.MeshInfoT()
    assert L.mpm_mesh_info(None, C.byref(info)) == _lib.MPM_EARG
    buf = C.create_string_buffer(256)
    L.mpm_last_error(buf, 256)
    assert b"null" in buf.value


def test_noalloc_capacity_constant_matches_header():
    """The binding's copy of the allocation-free solver's DOF limit is the header's."""
    from paper_2606_09275_amd import _lib
    m = re.search(r"#define\s+MPM_CG_NOALLOC_MAX_DOFS\s+(\d+)", HEADER.read_text())
    assert m and int(m.group(1)) == _lib.MPM_CG_NOALLOC_MAX_DOFS
