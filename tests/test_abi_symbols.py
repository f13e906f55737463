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
