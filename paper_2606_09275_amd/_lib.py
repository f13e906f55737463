"""ctypes declarations of the C ABI in include/mpm_gimp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "libmpmgimp.so"

MPM_OK, MPM_EARG, MPM_EDET, MPM_ESTENCIL, MPM_EOUTSIDE, MPM_ETREE, MPM_EHIP, MPM_ENONFINITE = 0, -1, -2, -3, -4, -5, -6, -7
MPM_F64, MPM_F32K = 0, 1
MPM_CG_NOALLOC_MAX_DOFS = 1635968  # largest n_dof of mpm_solve_cg_noalloc (static work space)


class RefineT(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("base", C.c_int32 * 3), ("h0", C.c_double), ("lvl_base", C.c_int32),
                ("lvl_max", C.c_int32), ("body_kind", C.c_int32), ("body", C.c_double * 8), ("dx_region", C.c_double),
                ("ghost", C.c_int32)]


class StateOutT(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("x", "l", "vol", "mass", "Jn", "bn", "Fn", "E", "nu", "sy")]


class MeshInfoT(C.Structure):
    _fields_ = [("n_leaf", C.c_int64), ("n_node", C.c_int64), ("n_hang", C.c_int64), ("n_dof", C.c_int64),
                ("nnz", C.c_int64), ("n_point", C.c_int64), ("n_straddle", C.c_int64),
                ("n_active_rows", C.c_int64), ("max_support", C.c_int32), ("lattice", C.c_int32 * 3),
                ("h_min", C.c_double), ("n_ghost_face", C.c_int64)]


class MeshArraysT(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("leaf", "node_ijk", "hang_ijk", "hang_support", "hang_weight",
                                          "hang_owner", "cell_nodes", "cell_cmat", "perm", "point_leaf",
                                          "point_nleaf", "row_ptr", "col")]


class StateT(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("x", "l", "vol", "mass", "Jn", "bn", "Fn", "E", "nu", "sy")] + \
               [("g", C.c_double * 3)]


class MPMError(RuntimeError):
    def __init__(self, code: int, msg: str, index: int):
        super().__init__(f"{msg} (status {code}, index {index})")
        self.code = code
        self.index = index


_lib = None


def lib():
    """Load the in-tree HIP library; fails loudly when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2606_09275_amd.build.build() "
                          "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    L = C.CDLL(str(LIB_PATH))
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.octree_build.restype = i32
    L.octree_build.argtypes = [C.POINTER(RefineT), vp, vp, i64, vp, C.POINTER(vp)]
    L.mpm_mesh_info.restype = i32
    L.mpm_mesh_info.argtypes = [vp, C.POINTER(MeshInfoT)]
    L.mpm_mesh_arrays.restype = i32
    L.mpm_mesh_arrays.argtypes = [vp, C.POINTER(MeshArraysT)]
    L.mpm_ghost_faces.restype = i32
    L.mpm_ghost_faces.argtypes = [vp, vp]
    L.mpm_mesh_free.restype = None
    L.mpm_mesh_free.argtypes = [vp]
    L.mpm_point_sort.restype = i32
    L.mpm_point_sort.argtypes = [vp, vp, i64, vp, vp, vp]
    L.mpm_permute.restype = i32
    L.mpm_permute.argtypes = [vp, vp, vp, vp, i32, vp]
    L.mpm_external_force.restype = i32
    L.mpm_external_force.argtypes = [vp, C.POINTER(StateT), vp, vp]
    L.mpm_assemble.restype = i32
    L.mpm_assemble.argtypes = [vp, C.POINTER(StateT), vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.mpm_assemble_adjoint.restype = i32
    L.mpm_assemble_adjoint.argtypes = [vp, C.POINTER(StateT), vp, vp, i32, vp, vp, vp, vp, vp]
    L.mpm_spmv.restype = i32
    L.mpm_spmv.argtypes = [vp, i32, vp, vp, vp, vp]
    L.mpm_solve_cg.restype = i32
    L.mpm_solve_cg.argtypes = [vp, i32, vp, vp, vp, vp, C.c_double, i32, C.POINTER(i32), C.POINTER(C.c_double), vp]
    L.mpm_solve_cg_noalloc.restype = i32
    L.mpm_solve_cg_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, C.c_double, i32, C.POINTER(i32),
                                       C.POINTER(C.c_double), vp]
    L.mpm_solve_gmres.restype = i32
    L.mpm_solve_gmres.argtypes = [vp, i32, vp, vp, vp, vp, C.c_double, i32, i32, C.POINTER(i32),
                                  C.POINTER(C.c_double), vp]
    L.mpm_assemble_dynamic.restype = i32
    L.mpm_assemble_dynamic.argtypes = [vp, C.POINTER(StateT), vp, vp, C.c_double, i32, vp, vp, vp, vp, vp, vp, vp,
                                       vp, vp, vp]
    L.mpm_split_mark.restype = i32
    L.mpm_split_mark.argtypes = [vp, vp, vp, i64, C.c_double, vp, C.POINTER(i64), vp]
    L.mpm_split_apply.restype = i32
    L.mpm_split_apply.argtypes = [vp, i64, vp, C.POINTER(StateT), vp, vp, vp, i32, C.POINTER(StateOutT), vp, vp,
                                  i64, vp]
    L.mpm_kernel_timing.restype = i32
    L.mpm_kernel_timing.argtypes = [vp, i32, vp]
    L.mpm_last_error.restype = i32
    L.mpm_last_error.argtypes = [C.c_char_p, C.c_size_t]
    L.mpm_last_error_index.restype = i64
    L.mpm_last_error_index.argtypes = []
    _lib = L
    return L


EXPORTED = ["octree_build", "mpm_mesh_info", "mpm_mesh_arrays", "mpm_ghost_faces", "mpm_mesh_free", "mpm_point_sort", "mpm_permute",
            "mpm_external_force", "mpm_assemble", "mpm_assemble_dynamic", "mpm_assemble_adjoint", "mpm_spmv",
            "mpm_solve_cg", "mpm_solve_cg_noalloc", "mpm_solve_gmres", "mpm_split_mark", "mpm_split_apply", "mpm_kernel_timing", "mpm_last_error",
            "mpm_last_error_index"]


def check(code: int):
    if code != MPM_OK:
        buf = C.create_string_buffer(512)
        lib().mpm_last_error(buf, 512)
        raise MPMError(code, buf.value.decode(errors="replace"), int(lib().mpm_last_error_index()))


_hip = None


def hip():
    """HIP runtime, used only to copy library-owned device arrays into caller tensors."""
    global _hip
    if _hip is None:
        for name in ("libamdhip64.so", "libamdhip64.so.7", "libamdhip64.so.6"):
            try:
                _hip = C.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
            _hip = C.CDLL(os.path.join(rocm, "lib", "libamdhip64.so"))
        _hip.hipMemcpy.restype = C.c_int
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    return _hip
