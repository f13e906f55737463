"""Python front end of the C ABI: torch tensors in, torch tensors out (marshalling only;
every step runs in the HIP library)."""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

import torch

from . import _lib
from ._lib import MPM_F32K, MPM_F64, check, lib

PRECISION = {"f64": MPM_F64, "fp64": MPM_F64, "f32k": MPM_F32K, "fp32k": MPM_F32K, MPM_F64: MPM_F64,
             MPM_F32K: MPM_F32K}
STATE_KEYS = ("x", "l", "vol", "mass", "Jn", "bn", "Fn", "E", "nu", "sy")
_D2D = 3


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def refine_struct(crit: dict, ghost: bool = False) -> _lib.RefineT:
    r = _lib.RefineT()
    r.lo = (C.c_double * 3)(*crit["lo"])
    r.base = (C.c_int32 * 3)(*crit["base"])
    r.h0 = crit["h0"]
    r.lvl_base = crit["lvl_base"]
    r.lvl_max = crit["lvl_max"]
    r.body_kind = crit["body_kind"]
    b = list(crit.get("body", ())) + [0.0] * (8 - len(crit.get("body", ())))
    r.body = (C.c_double * 8)(*b)
    r.dx_region = crit["dx_region"]
    r.ghost = 1 if ghost else 0
    return r


class Mesh:
    """Octree mesh + point order + CSR pattern, owned by the HIP library. ghost=True adds the
    ghost stabilisation of Section 4 to every assembly on the mesh."""

    def __init__(self, crit: dict, x: Optional[torch.Tensor] = None, l: Optional[torch.Tensor] = None,
                 ghost: bool = False):
        self._crit = refine_struct(crit, ghost)
        self.crit = dict(crit)
        h = C.c_void_p()
        n = 0 if x is None else int(x.shape[1])
        xp = lp = None
        if x is not None:
            x = x.contiguous()
            l = l.contiguous()
            xp = C.c_void_p(x.data_ptr()) if x.is_cuda else x.numpy().ctypes.data_as(C.c_void_p)
            lp = C.c_void_p(l.data_ptr()) if l.is_cuda else l.numpy().ctypes.data_as(C.c_void_p)
        check(lib().octree_build(C.byref(self._crit), xp, lp, n, _stream(), C.byref(h)))
        self.h = h
        inf = _lib.MeshInfoT()
        check(lib().mpm_mesh_info(self.h, C.byref(inf)))
        self.info = {k: (list(getattr(inf, k)) if k == "lattice" else getattr(inf, k)) for k, _ in inf._fields_}
        self._arrays = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                lib().mpm_mesh_free(h)
            except (AttributeError, TypeError, ImportError):
                pass  # interpreter shutdown: module globals already cleared; the process frees the GPU
            self.h = None

    # -------------------------------------------------------------- inspection
    def _copy(self, ptr, shape, dtype):
        out = torch.empty(shape, dtype=dtype, device="cuda")
        nbytes = out.numel() * out.element_size()
        if nbytes:
            torch.cuda.synchronize()
            rc = _lib.hip().hipMemcpy(C.c_void_p(out.data_ptr()), C.c_void_p(ptr), nbytes, _D2D)
            if rc != 0:
                raise RuntimeError(f"hipMemcpy failed ({rc})")
        return out

    def arrays(self) -> dict:
        if self._arrays is None:
            a = _lib.MeshArraysT()
            check(lib().mpm_mesh_arrays(self.h, C.byref(a)))
            i = self.info
            self._arrays = {
                "leaf": self._copy(a.leaf, (i["n_leaf"], 4), torch.int32),
                "node_ijk": self._copy(a.node_ijk, (i["n_node"], 3), torch.int32),
                "hang_ijk": self._copy(a.hang_ijk, (i["n_hang"], 3), torch.int32),
                "hang_support": self._copy(a.hang_support, (i["n_hang"], 4), torch.int32),
                "hang_weight": self._copy(a.hang_weight, (i["n_hang"], 4), torch.float64),
                "hang_owner": self._copy(a.hang_owner, (i["n_hang"],), torch.int32),
                "cell_nodes": self._copy(a.cell_nodes, (i["n_leaf"], 8), torch.int32),
                "cell_cmat": self._copy(a.cell_cmat, (i["n_leaf"], 8, 8), torch.float64),
                "perm": self._copy(a.perm, (i["n_point"],), torch.int64),
                "point_leaf": self._copy(a.point_leaf, (i["n_point"],), torch.int32),
                "point_nleaf": self._copy(a.point_nleaf, (i["n_point"],), torch.uint8),
                "row_ptr": self._copy(a.row_ptr, (i["n_dof"] + 1,), torch.int64),
                "col": self._copy(a.col, (i["nnz"],), torch.int32),
            }
        return self._arrays

    def ghost_faces(self) -> np.ndarray:
        """[n_ghost_face, 8] int32: lo leaf, hi leaf, axis, plane, b0, b1, c0, c1 (lattice units)."""
        out = np.zeros((self.info["n_ghost_face"], 8), dtype=np.int32)
        check(lib().mpm_ghost_faces(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    # -------------------------------------------------------------- point order
    def permute(self, src: torch.Tensor, perm: Optional[torch.Tensor] = None,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """[ncomp, n] (or [n]) original-order float64 device tensor -> sorted order (perm: the
        mesh's order when None)."""
        flat = src.dim() == 1
        s = src.reshape(1, -1) if flat else src
        s = s.contiguous().to(torch.float64)
        o = torch.empty_like(s) if out is None else out.reshape(s.shape)
        check(lib().mpm_permute(self.h, _ptr(perm), _ptr(s), _ptr(o), int(s.shape[0]), _stream()))
        return o.reshape(-1) if flat else o

    def point_sort(self, x: torch.Tensor, perm_out=None, leaf_out=None):
        n = int(x.shape[1])
        perm_out = torch.empty(n, dtype=torch.int64, device="cuda") if perm_out is None else perm_out
        leaf_out = torch.empty(n, dtype=torch.int32, device="cuda") if leaf_out is None else leaf_out
        check(lib().mpm_point_sort(self.h, _ptr(x.contiguous()), n, _ptr(perm_out), _ptr(leaf_out), _stream()))
        return perm_out, leaf_out

    def sorted_state(self, state: dict) -> dict:
        """Original-order state (numpy or torch, [ncomp, n]) -> sorted-order device tensors."""
        out = {}
        for k in STATE_KEYS:
            v = state.get(k)
            if v is None:
                continue
            t = torch.as_tensor(v, dtype=torch.float64).cuda()
            out[k] = self.permute(t)
        out["g"] = tuple(state.get("g", (0.0, 0.0, -9.81)))
        return out

    def kernel_timing(self, enable: int = -1):
        """enable 1/0 switches event timing of the assembly/gather/adjoint kernels; returns and
        resets (assembly ms, launches, adjoint ms, launches, gather ms, launches)."""
        buf = (C.c_double * 6)()
        check(lib().mpm_kernel_timing(self.h, int(enable), buf))
        return tuple(buf)

    # -------------------------------------------------------------- compute
    @staticmethod
    def _state(s: dict) -> _lib.StateT:
        st = _lib.StateT()
        for k in STATE_KEYS:
            t = s.get(k)
            setattr(st, k, None if t is None else _ptr(t).value)
        st.g = (C.c_double * 3)(*s.get("g", (0.0, 0.0, -9.81)))
        return st

    # -------------------------------------------------------------- GIMP refinement
    def split_mark(self, x: torch.Tensor, l: torch.Tensor, beta: float = 2.0, out: Optional[torch.Tensor] = None):
        """mpm_split_mark: uint8 flags [n] of the points to split and their count."""
        n = int(x.shape[1])
        flags = torch.empty(n, dtype=torch.uint8, device="cuda") if out is None else out
        cnt = C.c_int64(0)
        check(lib().mpm_split_mark(self.h, _ptr(x), _ptr(l), n, float(beta), _ptr(flags), C.byref(cnt), _stream()))
        return flags, int(cnt.value)

    SPLIT_FIELDS = {"x": 3, "l": 3, "vol": 1, "mass": 1, "Jn": 1, "bn": 6, "Fn": 9, "E": 1, "nu": 1, "sy": 1}

    def split_apply(self, s: dict, flags: torch.Tensor, n_split: int, X: Optional[torch.Tensor] = None,
                    v: Optional[torch.Tensor] = None, props: Optional[dict] = None) -> dict:
        """mpm_split_apply: new per-point arrays ([c][n_out] / [n_out]) of the fields present in s,
        plus "X" and "v" when given; props {"E"|"nu"|"sy": (a0, a1, a2, a3)} evaluates those
        parameters at the children's reference positions."""
        n = int(flags.shape[0])
        n_out = n + 7 * int(n_split)
        o = {}
        so = _lib.StateOutT()
        for k, c in self.SPLIT_FIELDS.items():
            if s.get(k) is None:
                continue
            shape = (c, n_out) if c > 1 else (n_out,)
            o[k] = torch.empty(shape, dtype=torch.float64, device="cuda")
            setattr(so, k, _ptr(o[k]).value)
        if X is not None:
            o["X"] = torch.empty((3, n_out), dtype=torch.float64, device="cuda")
        if v is not None:
            o["v"] = torch.empty((3, n_out), dtype=torch.float64, device="cuda")
        mask, coef = 0, [0.0] * 12
        for r, name in enumerate(("E", "nu", "sy")):
            if props and name in props:
                mask |= 1 << r
                coef[4 * r:4 * r + 4] = [float(a) for a in props[name]]
        cbuf = (C.c_double * 12)(*coef)
        st = self._state(s)
        check(lib().mpm_split_apply(self.h, n, _ptr(flags), C.byref(st), _ptr(X), _ptr(v), cbuf, mask, C.byref(so),
                                    _ptr(o.get("X")), _ptr(o.get("v")), n_out, _stream()))
        return o

    def external_force(self, s: dict, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = torch.empty(self.info["n_dof"], dtype=torch.float64, device="cuda") if out is None else out
        st = self._state(s)
        check(lib().mpm_external_force(self.h, C.byref(st), _ptr(out), _stream()))
        return out

    def assemble(self, s: dict, u: torch.Tensor, precision="f64", f_ext=None, dirichlet=None, want_K=True,
                 want_sigma=True, want_residual=True, commit=False, out: Optional[dict] = None) -> dict:
        p = PRECISION.get(precision, precision)
        i = self.info
        n = i["n_point"]
        o = {} if out is None else out
        dev = "cuda"
        if "f_int" not in o:
            o["f_int"] = torch.empty(i["n_dof"], dtype=torch.float64, device=dev)
        if want_K and "K" not in o:
            o["K"] = torch.empty(i["nnz"], dtype=torch.float64 if p == MPM_F64 else torch.float32, device=dev)
        if want_sigma and "sigma" not in o:
            o["sigma"] = torch.empty((6, n), dtype=torch.float64, device=dev)
        if want_residual:
            o.setdefault("r", torch.empty(i["n_dof"], dtype=torch.float64, device=dev))
            o.setdefault("rnorm", torch.empty(1, dtype=torch.float64, device=dev))
        if commit:
            o.setdefault("F_new", torch.empty((9, n), dtype=torch.float64, device=dev))
            o.setdefault("be_new", torch.empty((6, n), dtype=torch.float64, device=dev))
        st = self._state(s)
        check(lib().mpm_assemble(self.h, C.byref(st), _ptr(u), p, _ptr(f_ext), _ptr(dirichlet), _ptr(o["f_int"]),
                                 _ptr(o.get("K") if want_K else None), _ptr(o.get("sigma") if want_sigma else None),
                                 _ptr(o.get("r") if want_residual else None),
                                 _ptr(o.get("rnorm") if want_residual else None),
                                 _ptr(o.get("F_new") if commit else None), _ptr(o.get("be_new") if commit else None),
                                 _stream()))
        return o

    def assemble_dynamic(self, s: dict, u: torch.Tensor, v_n: torch.Tensor, dt: float, precision="f64", f_ext=None,
                         dirichlet=None, want_K=True, want_sigma=True, want_residual=True, want_kinematics=False,
                         out: Optional[dict] = None) -> dict:
        """mpm_assemble_dynamic: f_int (internal + Newmark inertia force), K (+ 2/dt^2 consistent
        mass), sigma, residual; v_n [3][n] sorted-order point velocities; optional point
        accelerations `a_new` and velocities `v_new` [3][n]."""
        p = PRECISION.get(precision, precision)
        i = self.info
        n = i["n_point"]
        o = {} if out is None else out
        dev = "cuda"
        if "f_int" not in o:
            o["f_int"] = torch.empty(i["n_dof"], dtype=torch.float64, device=dev)
        if want_K and "K" not in o:
            o["K"] = torch.empty(i["nnz"], dtype=torch.float64 if p == MPM_F64 else torch.float32, device=dev)
        if want_sigma and "sigma" not in o:
            o["sigma"] = torch.empty((6, n), dtype=torch.float64, device=dev)
        if want_residual:
            o.setdefault("r", torch.empty(i["n_dof"], dtype=torch.float64, device=dev))
            o.setdefault("rnorm", torch.empty(1, dtype=torch.float64, device=dev))
        if want_kinematics:
            o.setdefault("a_new", torch.empty((3, n), dtype=torch.float64, device=dev))
            o.setdefault("v_new", torch.empty((3, n), dtype=torch.float64, device=dev))
        st = self._state(s)
        check(lib().mpm_assemble_dynamic(self.h, C.byref(st), _ptr(u), _ptr(v_n.contiguous()), float(dt), p,
                                         _ptr(f_ext), _ptr(dirichlet), _ptr(o["f_int"]),
                                         _ptr(o.get("K") if want_K else None),
                                         _ptr(o.get("sigma") if want_sigma else None),
                                         _ptr(o.get("r") if want_residual else None),
                                         _ptr(o.get("rnorm") if want_residual else None),
                                         _ptr(o.get("a_new") if want_kinematics else None),
                                         _ptr(o.get("v_new") if want_kinematics else None), _stream()))
        return o

    def spmv(self, K: torch.Tensor, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """y = K x on the mesh's CSR (K FP64 or FP32, x FP64)."""
        p = MPM_F64 if K.dtype == torch.float64 else MPM_F32K
        y = torch.empty_like(x) if out is None else out
        check(lib().mpm_spmv(self.h, p, _ptr(K), _ptr(x), _ptr(y), _stream()))
        return y

    def solve_cg(self, K: torch.Tensor, b: torch.Tensor, dirichlet=None, rtol: float = 1e-8, max_iter: int = 1000,
                 out: Optional[torch.Tensor] = None):
        """Jacobi-preconditioned CG for K_ff x_f = b_f (free DOFs); returns (x, iterations, relres)."""
        p = MPM_F64 if K.dtype == torch.float64 else MPM_F32K
        x = torch.empty_like(b) if out is None else out
        it = C.c_int32(0)
        rr = C.c_double(0.0)
        check(lib().mpm_solve_cg(self.h, p, _ptr(K), _ptr(dirichlet), _ptr(b), _ptr(x), float(rtol), int(max_iter),
                                 C.byref(it), C.byref(rr), _stream()))
        return x, int(it.value), float(rr.value)

    def solve_gmres(self, K: torch.Tensor, b: torch.Tensor, dirichlet=None, rtol: float = 1e-8, restart: int = 30,
                    max_iter: int = 1000, out: Optional[torch.Tensor] = None):
        """Restarted GMRES with the Jacobi preconditioner on the right for K_ff x_f = b_f (free
        DOFs); returns (x, Arnoldi steps, true relative residual)."""
        p = MPM_F64 if K.dtype == torch.float64 else MPM_F32K
        x = torch.empty_like(b) if out is None else out
        it = C.c_int32(0)
        rr = C.c_double(0.0)
        check(lib().mpm_solve_gmres(self.h, p, _ptr(K), _ptr(dirichlet), _ptr(b), _ptr(x), float(rtol), int(restart),
                                    int(max_iter), C.byref(it), C.byref(rr), _stream()))
        return x, int(it.value), float(rr.value)

    def adjoint(self, s: dict, u: torch.Tensor, lam: torch.Tensor, precision="f64", out: Optional[dict] = None):
        p = PRECISION.get(precision, precision)
        n = self.info["n_point"]
        o = {} if out is None else out
        for k in ("dE", "dnu", "dsy", "dV"):
            if k not in o:
                o[k] = torch.empty(n, dtype=torch.float64, device="cuda")
        st = self._state(s)
        check(lib().mpm_assemble_adjoint(self.h, C.byref(st), _ptr(u), _ptr(lam), p, _ptr(o["dE"]), _ptr(o["dnu"]),
                                         _ptr(o["dsy"]), _ptr(o["dV"]), _stream()))
        return o
