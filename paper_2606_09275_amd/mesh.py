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


# number of components of each per-point state field ([c][n] SoA, float64)
STATE_COMPONENTS = {"x": 3, "l": 3, "vol": 1, "mass": 1, "Jn": 1, "bn": 6, "Fn": 9, "E": 1, "nu": 1, "sy": 1}


def _validate(specs):
    """Reject tensors the library would misread, before anything is launched: the kernels
    take raw pointers and trust the sizes the mesh implies, so a float32 tensor read as
    float64, or a short one, would be read past its end. specs: (tensor or None, name,
    element count or None, allowed dtypes). Every dtype and size is checked before any layout
    or device, so that the first two checks also hold for host tensors."""
    specs = [sp for sp in specs if sp[0] is not None]
    for t, name, numel, dtypes in specs:
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
        if t.dtype not in dtypes:
            raise ValueError(f"{name}: expected dtype {' or '.join(str(d) for d in dtypes)}, got {t.dtype}")
        if numel is not None and t.numel() != numel:
            raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    for t, name, _, _ in specs:
        if not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous tensor")
    for t, name, _, _ in specs:
        if not t.is_cuda:
            raise ValueError(f"{name}: expected a device tensor")


F64 = (torch.float64,)


def _check(t, name: str, numel: Optional[int] = None, dtypes=F64):
    _validate([(t, name, numel, dtypes)])


def state_specs(s: dict, n: int):
    return [(s.get(k), f"state[{k!r}]", c * n, F64) for k, c in STATE_COMPONENTS.items()]


def check_state(s: dict, n: int):
    """Validate the per-point fields present in s for n points (float64, [c][n] or [n])."""
    _validate(state_specs(s, n))


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
        n = int(s.shape[1])
        if perm is None and n != self.info["n_point"]:
            raise ValueError(f"permute: expected {self.info['n_point']} points per component, got {n}")
        _check(perm, "perm", n, (torch.int64,))
        _check(s, "src", s.numel())
        if out is not None:
            _check(out, "out", s.numel())
        o = torch.empty_like(s) if out is None else out.reshape(s.shape)
        check(lib().mpm_permute(self.h, _ptr(perm), _ptr(s), _ptr(o), int(s.shape[0]), _stream()))
        return o.reshape(-1) if flat else o

    def point_sort(self, x: torch.Tensor, perm_out=None, leaf_out=None):
        n = int(x.shape[1])
        _check(x.contiguous(), "x", 3 * n)
        perm_out = torch.empty(n, dtype=torch.int64, device="cuda") if perm_out is None else perm_out
        leaf_out = torch.empty(n, dtype=torch.int32, device="cuda") if leaf_out is None else leaf_out
        _check(perm_out, "perm_out", n, (torch.int64,))
        _check(leaf_out, "leaf_out", n, (torch.int32,))
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
    def _state(s: dict, n: Optional[int] = None) -> _lib.StateT:
        if n is not None:
            check_state(s, n)
        st = _lib.StateT()
        for k in STATE_KEYS:
            t = s.get(k)
            setattr(st, k, None if t is None else _ptr(t).value)
        st.g = (C.c_double * 3)(*s.get("g", (0.0, 0.0, -9.81)))
        return st

    def _K_spec(self, K):
        return (K, "K", self.info["nnz"], (torch.float64, torch.float32))

    def _check_io(self, s: dict, u, f_ext, dirichlet, o: dict, precision: int, extra=()):
        """Sizes and dtypes of the assembly's state, vectors and given outputs (_validate)."""
        i = self.info
        n, nd = i["n_point"], i["n_dof"]
        kt = torch.float64 if precision == MPM_F64 else torch.float32
        specs = [(u, "u", nd, F64), (f_ext, "f_ext", nd, F64), (dirichlet, "dirichlet", nd, (torch.uint8, torch.bool)),
                 (o.get("f_int"), "f_int", nd, F64), (o.get("K"), "K", i["nnz"], (kt,)),
                 (o.get("r"), "r", nd, F64), (o.get("rnorm"), "rnorm", 1, F64)]
        specs += [(o.get(k), k, c * n, F64) for k, c in (("sigma", 6), ("F_new", 9), ("be_new", 6), ("a_new", 3),
                                                          ("v_new", 3))]
        _validate(specs + list(extra) + state_specs(s, n))

    # -------------------------------------------------------------- GIMP refinement
    def split_mark(self, x: torch.Tensor, l: torch.Tensor, beta: float = 2.0, out: Optional[torch.Tensor] = None):
        """mpm_split_mark: uint8 flags [n] of the points to split and their count."""
        n = int(x.shape[1])
        _check(x, "x", 3 * n)
        _check(l, "l", 3 * n)
        flags = torch.empty(n, dtype=torch.uint8, device="cuda") if out is None else out
        _check(flags, "out", n, (torch.uint8,))
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
        _check(flags, "flags", n, (torch.uint8,))
        _check(X, "X", 3 * n)
        _check(v, "v", 3 * n)
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
        st = self._state(s, n)
        check(lib().mpm_split_apply(self.h, n, _ptr(flags), C.byref(st), _ptr(X), _ptr(v), cbuf, mask, C.byref(so),
                                    _ptr(o.get("X")), _ptr(o.get("v")), n_out, _stream()))
        return o

    def external_force(self, s: dict, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = torch.empty(self.info["n_dof"], dtype=torch.float64, device="cuda") if out is None else out
        _check(out, "out", self.info["n_dof"])
        st = self._state(s, self.info["n_point"])
        check(lib().mpm_external_force(self.h, C.byref(st), _ptr(out), _stream()))
        return out

    def assemble(self, s: dict, u: torch.Tensor, precision="f64", f_ext=None, dirichlet=None, want_K=True,
                 want_sigma=True, want_residual=True, commit=False, out: Optional[dict] = None) -> dict:
        p = PRECISION.get(precision, precision)
        i = self.info
        n = i["n_point"]
        o = {} if out is None else out
        self._check_io(s, u, f_ext, dirichlet, o, p)
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
        self._check_io(s, u, f_ext, dirichlet, o, p, extra=[(v_n.contiguous(), "v_n", 3 * n, F64)])
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
        nd = self.info["n_dof"]
        _validate([self._K_spec(K), (x, "x", nd, F64), (out, "out", nd, F64)])
        y = torch.empty_like(x) if out is None else out
        check(lib().mpm_spmv(self.h, p, _ptr(K), _ptr(x), _ptr(y), _stream()))
        return y

    def solve_cg(self, K: torch.Tensor, b: torch.Tensor, dirichlet=None, rtol: float = 1e-8, max_iter: int = 1000,
                 out: Optional[torch.Tensor] = None, noalloc: bool = False):
        """Jacobi-preconditioned CG for K_ff x_f = b_f (free DOFs); returns (x, iterations, relres).
        noalloc=True calls mpm_solve_cg_noalloc (static work space, no device allocation; n_dof
        at most MPM_CG_NOALLOC_MAX_DOFS; pass `out` to allocate nothing here either)."""
        p = MPM_F64 if K.dtype == torch.float64 else MPM_F32K
        nd = self.info["n_dof"]
        _validate([self._K_spec(K), (b, "b", nd, F64), (dirichlet, "dirichlet", nd, (torch.uint8, torch.bool)),
                   (out, "out", nd, F64)])
        x = torch.empty_like(b) if out is None else out
        it = C.c_int32(0)
        rr = C.c_double(0.0)
        fn = lib().mpm_solve_cg_noalloc if noalloc else lib().mpm_solve_cg
        check(fn(self.h, p, _ptr(K), _ptr(dirichlet), _ptr(b), _ptr(x), float(rtol), int(max_iter), C.byref(it),
                 C.byref(rr), _stream()))
        return x, int(it.value), float(rr.value)

    def solve_gmres(self, K: torch.Tensor, b: torch.Tensor, dirichlet=None, rtol: float = 1e-8, restart: int = 30,
                    max_iter: int = 1000, out: Optional[torch.Tensor] = None):
        """Restarted GMRES with the Jacobi preconditioner on the right for K_ff x_f = b_f (free
        DOFs); returns (x, Arnoldi steps, true relative residual)."""
        p = MPM_F64 if K.dtype == torch.float64 else MPM_F32K
        nd = self.info["n_dof"]
        _validate([self._K_spec(K), (b, "b", nd, F64), (dirichlet, "dirichlet", nd, (torch.uint8, torch.bool)),
                   (out, "out", nd, F64)])
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
        _validate([(u, "u", self.info["n_dof"], F64), (lam, "lambda", self.info["n_dof"], F64)] +
                  [(o.get(k), k, n, F64) for k in ("dE", "dnu", "dsy", "dV")] + state_specs(s, n))
        for k in ("dE", "dnu", "dsy", "dV"):
            if k not in o:
                o[k] = torch.empty(n, dtype=torch.float64, device="cuda")
        st = self._state(s)
        check(lib().mpm_assemble_adjoint(self.h, C.byref(st), _ptr(u), _ptr(lam), p, _ptr(o["dE"]), _ptr(o["dnu"]),
                                         _ptr(o["dsy"]), _ptr(o["dV"]), _stream()))
        return o
