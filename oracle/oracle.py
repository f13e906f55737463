"""ctypes front end of the CPU oracle (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import this module.
The library (paper_2606_09275_amd) never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
LIB = HERE / "liboracle.so"
SOURCES = ["orc_mesh.c", "orc_point.c", "orc_ghost.c", "orc_split.c"]

_i64 = np.int64
_f64 = np.float64


def build(verbose: bool = False) -> Path:
    """Compile the oracle with gcc (plain C11, FP64, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp", "-Wall",
           "-Wno-unused-function",
           "-o", str(LIB)] + [str(HERE / s) for s in SOURCES] + ["-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + r.stderr)
    if verbose and r.stderr:
        print(r.stderr)
    return LIB


class _Crit(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("base", C.c_int32 * 3), ("h0", C.c_double), ("lvl_base", C.c_int32),
                ("lvl_max", C.c_int32), ("body_kind", C.c_int32), ("body", C.c_double * 8), ("dx_region", C.c_double)]


class _State(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("x", "l", "vol", "mass", "Jn", "bn", "E", "nu", "sy", "Fn")] + \
               [("g", C.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB.exists():
            build()
        L = C.CDLL(str(LIB))
        vp, i64p = C.c_void_p, C.POINTER(C.c_int64)
        L.orc_mesh_build.restype = C.c_void_p
        L.orc_mesh_build.argtypes = [C.POINTER(_Crit), C.POINTER(C.c_int32)]
        L.orc_mesh_free.argtypes = [vp]
        L.orc_mesh_counts.argtypes = [vp, vp]
        for f in ("orc_mesh_leaves", "orc_mesh_nodes"):
            getattr(L, f).argtypes = [vp, vp]
        L.orc_mesh_hanging.argtypes = [vp, vp, vp, vp, vp]
        L.orc_mesh_cells.argtypes = [vp, vp, vp, vp]
        L.orc_mesh_set_points.restype = C.c_int32
        L.orc_mesh_set_points.argtypes = [vp, vp, vp, C.c_int64, i64p]
        L.orc_mesh_perm.argtypes = [vp, vp, vp, vp]
        L.orc_mesh_csr.argtypes = [vp, vp, vp]
        L.orc_point_basis.restype = C.c_int32
        L.orc_point_basis.argtypes = [vp, vp, vp, vp, vp, vp]
        L.orc_material_point.restype = C.c_int32
        L.orc_material_point.argtypes = [vp, vp, C.c_double, C.c_double, C.c_double, C.c_double, vp, vp, vp, vp, vp]
        L.orc_assemble.restype = C.c_int32
        L.orc_assemble.argtypes = [vp, C.POINTER(_State), vp, vp, vp, vp, vp, vp, vp, vp, i64p]
        L.orc_assemble_threads.restype = C.c_int32
        L.orc_assemble_threads.argtypes = [vp, C.POINTER(_State), vp, vp, vp, vp, C.c_int32, i64p]
        L.orc_external_force.restype = C.c_int32
        L.orc_external_force.argtypes = [vp, C.POINTER(_State), vp]
        L.orc_mesh_set_ghost.argtypes = [vp, C.c_int32]
        L.orc_ghost_nfaces.restype = C.c_int64
        L.orc_ghost_nfaces.argtypes = [vp]
        L.orc_ghost_faces.argtypes = [vp, vp]
        L.orc_ghost_assemble.restype = C.c_int32
        L.orc_ghost_assemble.argtypes = [vp, C.POINTER(_State), vp, vp, vp, vp]
        L.orc_split_mark.restype = C.c_int32
        L.orc_split_mark.argtypes = [vp, vp, vp, C.c_int64, C.c_double, vp, i64p]
        L.orc_inertia.restype = C.c_int32
        L.orc_inertia.argtypes = [vp, C.POINTER(_State), vp, vp, C.c_double, vp, vp, vp, vp, i64p]
        L.orc_residual.argtypes = [C.c_int64, vp, vp, vp, vp, vp]
        L.orc_adjoint.restype = C.c_int32
        L.orc_adjoint.argtypes = [vp, C.POINTER(_State), vp, vp, vp, vp, vp, vp, i64p]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code, index=-1):
        super().__init__(f"oracle status {code} (index {index})")
        self.code = code
        self.index = index


def make_crit(d: dict) -> _Crit:
    c = _Crit()
    c.lo = (C.c_double * 3)(*d["lo"])
    c.base = (C.c_int32 * 3)(*d["base"])
    c.h0 = d["h0"]
    c.lvl_base = d["lvl_base"]
    c.lvl_max = d["lvl_max"]
    c.body_kind = d["body_kind"]
    c.body = (C.c_double * 8)(*(list(d["body"]) + [0.0] * (8 - len(d["body"]))))
    c.dx_region = d["dx_region"]
    return c


MAXI = 27


class OracleMesh:
    def __init__(self, crit: dict, ghost: bool = False):
        self._crit = make_crit(crit)
        st = C.c_int32(0)
        self.h = lib().orc_mesh_build(C.byref(self._crit), C.byref(st))
        if not self.h:
            raise OracleError(st.value)
        self._keep = []
        lib().orc_mesh_set_ghost(self.h, 1 if ghost else 0)

    def ghost_faces(self) -> np.ndarray:
        """Ghost faces (lo leaf, hi leaf, axis, plane, b0, b1, c0, c1), lattice units."""
        n = int(lib().orc_ghost_nfaces(self.h))
        out = np.zeros((n, 8), np.int32)
        if n:
            lib().orc_ghost_faces(self.h, _p(out))
        return out

    def ghost(self, s: dict, u: np.ndarray) -> dict:
        """Ghost term: K_G on the CSR pattern, f_G = K_G u, per-leaf maximum Young's modulus."""
        c = self.counts()
        st = self._state(s)
        u = np.ascontiguousarray(u, dtype=_f64)
        K = np.zeros(c["nnz"], _f64)
        f = np.zeros(3 * c["n_node"], _f64)
        beta = np.zeros(c["n_leaf"], _f64)
        code = lib().orc_ghost_assemble(self.h, C.byref(st), _p(u), _p(K), _p(f), _p(beta))
        if code != 0:
            raise OracleError(code)
        return dict(K=K, f=f, beta=beta)

    def split_mark(self, x: np.ndarray, l: np.ndarray, beta: float = 2.0) -> np.ndarray:
        """GIMP refinement criterion (Section 5) for points x, l [3][n] (any order): uint8 flags."""
        x = np.ascontiguousarray(x, dtype=_f64)
        l = np.ascontiguousarray(l, dtype=_f64)
        out = np.zeros(x.shape[1], np.uint8)
        bad = C.c_int64(-1)
        code = lib().orc_split_mark(self.h, _p(x), _p(l), x.shape[1], float(beta), _p(out), C.byref(bad))
        if code != 0:
            raise OracleError(code, bad.value)
        return out

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_mesh_free(self.h)
            self.h = None

    def counts(self) -> dict:
        out = np.zeros(9, dtype=_i64)
        lib().orc_mesh_counts(self.h, _p(out))
        keys = ["n_leaf", "n_node_all", "n_node", "n_hang", "n_point", "nnz", "n_straddle", "max_support",
                "n_active_rows"]
        return dict(zip(keys, (int(v) for v in out)))

    def leaves(self) -> np.ndarray:
        out = np.zeros((self.counts()["n_leaf"], 4), dtype=np.int32)
        lib().orc_mesh_leaves(self.h, _p(out))
        return out

    def nodes(self) -> np.ndarray:
        out = np.zeros((self.counts()["n_node"], 3), dtype=np.int32)
        lib().orc_mesh_nodes(self.h, _p(out))
        return out

    def hanging(self):
        nh = self.counts()["n_hang"]
        ijk = np.zeros((nh, 3), np.int32)
        sup = np.zeros((nh, 4), np.int32)
        w = np.zeros((nh, 4), _f64)
        own = np.zeros(nh, np.int32)
        lib().orc_mesh_hanging(self.h, _p(ijk), _p(sup), _p(w), _p(own))
        return ijk, sup, w, own

    def cells(self):
        nl = self.counts()["n_leaf"]
        n = np.zeros(nl, np.int32)
        ids = np.zeros((nl, MAXI), np.int32)
        cm = np.zeros((nl, 8, MAXI), _f64)
        lib().orc_mesh_cells(self.h, _p(n), _p(ids), _p(cm))
        return n, ids, cm

    def set_points(self, x: np.ndarray, l: np.ndarray):
        x = np.ascontiguousarray(x, dtype=_f64)
        l = np.ascontiguousarray(l, dtype=_f64)
        bad = C.c_int64(-1)
        st = lib().orc_mesh_set_points(self.h, _p(x), _p(l), x.shape[1], C.byref(bad))
        if st != 0:
            raise OracleError(st, bad.value)
        self.n_point = x.shape[1]

    def _need_points(self, what):
        if getattr(self, "n_point", None) is None:
            raise RuntimeError(f"OracleMesh.{what}: call set_points first (the order and the pattern depend on them)")

    def perm(self):
        self._need_points("perm")
        n = self.n_point
        perm = np.zeros(n, _i64)
        pl = np.zeros(n, np.int32)
        nl = np.zeros(n, np.uint8)
        lib().orc_mesh_perm(self.h, _p(perm), _p(pl), _p(nl))
        return perm, pl, nl

    def csr(self):
        self._need_points("csr")
        c = self.counts()
        rp = np.zeros(3 * c["n_node"] + 1, _i64)
        col = np.zeros(c["nnz"], np.int32)
        lib().orc_mesh_csr(self.h, _p(rp), _p(col))
        return rp, col

    def point_basis(self, x, l):
        x = np.ascontiguousarray(x, dtype=_f64)
        l = np.ascontiguousarray(l, dtype=_f64)
        node = np.zeros(128, np.int32)
        S = np.zeros(128, _f64)
        dS = np.zeros((128, 3), _f64)
        ns = lib().orc_point_basis(self.h, _p(x), _p(l), _p(node), _p(S), _p(dS))
        if ns < 0:
            raise OracleError(ns)
        return node[:ns].copy(), S[:ns].copy(), dS[:ns].copy()

    def _state(self, s: dict, g=(0.0, 0.0, -9.81)) -> _State:
        st = _State()
        arrs = {}
        for k in ("x", "l", "vol", "mass", "Jn", "bn", "E", "nu", "sy", "Fn"):
            if k in s and s[k] is not None:
                arrs[k] = np.ascontiguousarray(s[k], dtype=_f64)
                setattr(st, k, arrs[k].ctypes.data)
        st.g = (C.c_double * 3)(*s.get("g", g))
        self._keep = arrs
        return st

    def assemble(self, s: dict, u: np.ndarray, want_K: bool = True) -> dict:
        c = self.counts()
        n = self.n_point
        st = self._state(s)
        u = np.ascontiguousarray(u, dtype=_f64)
        f = np.zeros(3 * c["n_node"], _f64)
        K = np.zeros(c["nnz"], _f64) if want_K else None
        sig = np.zeros((6, n), _f64)
        Fnew = np.zeros((9, n), _f64) if s.get("Fn") is not None else None
        be = np.zeros((6, n), _f64)
        pl = np.zeros(n, np.uint8)
        q = np.zeros(n, _f64)
        bad = C.c_int64(-1)
        code = lib().orc_assemble(self.h, C.byref(st), _p(u), _p(f), _p(K), _p(sig), _p(Fnew), _p(be), _p(pl),
                                  _p(q), C.byref(bad))
        if code != 0:
            raise OracleError(code, bad.value)
        return dict(f_int=f, K=K, sigma=sig, Fnew=Fnew, be=be, plastic=pl, q_trial=q)

    def assemble_threads(self, s: dict, u: np.ndarray, nthreads: int, want_K: bool = True) -> dict:
        """orc_assemble on nthreads host threads (f_int, K, sigma; per-thread sums added in
        thread order). For timing the oracle on all cores."""
        c = self.counts()
        n = self.n_point
        st = self._state(s)
        u = np.ascontiguousarray(u, dtype=_f64)
        f = np.zeros(3 * c["n_node"], _f64)
        K = np.zeros(c["nnz"], _f64) if want_K else None
        sig = np.zeros((6, n), _f64)
        bad = C.c_int64(-1)
        code = lib().orc_assemble_threads(self.h, C.byref(st), _p(u), _p(f), _p(K), _p(sig), int(nthreads),
                                          C.byref(bad))
        if code != 0:
            raise OracleError(code, bad.value)
        return dict(f_int=f, K=K, sigma=sig)

    def external_force(self, s: dict) -> np.ndarray:
        st = self._state(s)
        f = np.zeros(3 * self.counts()["n_node"], _f64)
        code = lib().orc_external_force(self.h, C.byref(st), _p(f))
        if code != 0:
            raise OracleError(code)
        return f

    def inertia(self, s: dict, u: np.ndarray, vel: np.ndarray, dt: float, want_K: bool = True) -> dict:
        """Newmark (gamma = 1, beta = 1/2) inertia force, (2/dt^2) x consistent mass on the CSR
        pattern, point accelerations and updated velocities ([3][n], original order)."""
        c = self.counts()
        n = self.n_point
        st = self._state(s)
        u = np.ascontiguousarray(u, dtype=_f64)
        vel = np.ascontiguousarray(vel, dtype=_f64)
        f = np.zeros(3 * c["n_node"], _f64)
        K = np.zeros(c["nnz"], _f64) if want_K else None
        a = np.zeros((3, n), _f64)
        v = np.zeros((3, n), _f64)
        bad = C.c_int64(-1)
        code = lib().orc_inertia(self.h, C.byref(st), _p(u), _p(vel), C.c_double(dt), _p(f), _p(K), _p(a), _p(v),
                                 C.byref(bad))
        if code != 0:
            raise OracleError(code, bad.value)
        return dict(f_iner=f, K_mass=K, a=a, v=v)

    def adjoint(self, s: dict, u: np.ndarray, lam: np.ndarray) -> dict:
        n = self.n_point
        st = self._state(s)
        u = np.ascontiguousarray(u, dtype=_f64)
        lam = np.ascontiguousarray(lam, dtype=_f64)
        out = {k: np.zeros(n, _f64) for k in ("dE", "dnu", "dsy", "dV")}
        bad = C.c_int64(-1)
        code = lib().orc_adjoint(self.h, C.byref(st), _p(u), _p(lam), _p(out["dE"]), _p(out["dnu"]),
                                 _p(out["dsy"]), _p(out["dV"]), C.byref(bad))
        if code != 0:
            raise OracleError(code, bad.value)
        return out


def material_point(dF, bn6, Jn, E, nu, sy, want_tangent=True) -> dict:
    dF = np.ascontiguousarray(np.asarray(dF, dtype=_f64).reshape(9))
    bn6 = np.ascontiguousarray(np.asarray(bn6, dtype=_f64).reshape(6))
    sig, tau, be, info = np.zeros(6), np.zeros(6), np.zeros(6), np.zeros(3)
    a = np.zeros(81) if want_tangent else None
    code = lib().orc_material_point(_p(dF), _p(bn6), float(Jn), float(E), float(nu), float(sy), _p(sig), _p(tau),
                                    _p(a), _p(be), _p(info))
    if code != 0:
        raise OracleError(code)
    return dict(sigma=sig, tau=tau, a=None if a is None else a.reshape(3, 3, 3, 3), be=be,
                plastic=bool(info[0]), q_trial=info[1], J=info[2])


def residual(f_int, f_ext, dirichlet):
    f_int = np.ascontiguousarray(f_int, dtype=_f64)
    f_ext = None if f_ext is None else np.ascontiguousarray(f_ext, dtype=_f64)
    d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
    r = np.zeros_like(f_int)
    rn = C.c_double(0)
    lib().orc_residual(f_int.size, _p(f_int), _p(f_ext), _p(d), _p(r), C.byref(rn))
    return r, rn.value
