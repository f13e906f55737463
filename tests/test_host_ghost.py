"""Host part of the ghost stabilisation (Section 4) on CPU through a test shim: the library's
ghost-face builder, given the oracle's tree (leaves, I(K) and C_K), finds the oracle's ghost
faces bit for bit, and its per-face jump matrices (2 x 2 Gauss rule) reproduce the oracle's
penalty (3 x 3 Gauss rule, assembled into the CSR) as a quadratic form u . K_G u on random
displacements, on meshes with hanging nodes, jittered points and a varying Young's modulus.
No GPU call is made."""
import ctypes as C
import subprocess
from pathlib import Path

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle.oracle import OracleMesh
from tests.helpers import morton3_np, tiny_workload

ROOT = Path(__file__).resolve().parent.parent
SHIM_SRC = ROOT / "tests" / "shim" / "host_tree_shim.cpp"
SHIM = ROOT / "tests" / "shim" / "libhostghost.so"
_lib = None


def shim():
    global _lib
    if _lib is None:
        srcs = [SHIM_SRC, ROOT / "paper_2606_09275_amd" / "csrc" / "ghost_host.cpp"]
        deps = srcs + [ROOT / "paper_2606_09275_amd" / "csrc" / h for h in ("internal.h", "geom.h")]
        stale = not SHIM.exists() or any(s.stat().st_mtime > SHIM.stat().st_mtime for s in deps)
        if stale:
            cmd = ["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", "-x", "c++",
                   "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + [str(s) for s in srcs] + ["-o", str(SHIM)]
            r = subprocess.run(cmd, capture_output=True, text=True)
            assert r.returncode == 0, r.stderr
        _lib = C.CDLL(str(SHIM))
        _lib.shim_ghost.restype = C.c_int64
        _lib.shim_ghost.argtypes = [C.c_int64] + [C.c_void_p] * 5 + [C.c_double, C.c_int32, C.c_void_p, C.c_void_p]
    return _lib


def _tree(w, o):
    """The oracle's tree in the layout of the library's host arrays: every leaf of a balanced
    tree has exactly 8 independent nodes in I(K)."""
    lv = np.ascontiguousarray(o.leaves(), np.int32)
    n, ids, cm = o.cells()
    assert np.all(n == 8)
    keys = np.ascontiguousarray(morton3_np(lv[:, 0], lv[:, 1], lv[:, 2]), np.uint64)
    return dict(leaf=lv, key=keys, nodes=np.ascontiguousarray(ids[:, :8], np.int32),
                cmat=np.ascontiguousarray(cm[:, :, :8], np.float64))


def _case(kind, jit):
    if kind == "c0":
        w = W.get("c0")
    else:
        w = tiny_workload(kind, E=1e4)
        w.keep = lambda x, y, z: z < 0.55
    o = OracleMesh(w.crit(), ghost=True)
    lv = o.leaves()
    ps = W.make_points(w, lv[:, :3], lv[:, 3])
    if jit is not None:
        ps = W.jitter_points(w, ps, jit)
    o.set_points(ps.x, ps.l)
    st = W.make_state(w, ps)
    if kind != "c0":
        st["E"] = w.E * (1.0 + ps.x[0] + 0.5 * ps.x[1] ** 2)
    return w, o, st


def _host_ghost(w, o, pop):
    t = _tree(w, o)
    pop = np.ascontiguousarray(pop, np.uint8)
    lo = np.ascontiguousarray(w.lo, np.float64)
    lat = np.ascontiguousarray(w.lattice_dims(), np.int32)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    nf = int(shim().shim_ghost(t["leaf"].shape[0], p(t["leaf"]), p(t["key"]), p(t["nodes"]), p(t["cmat"]), p(lo),
                               w.h_min, w.lvl_max, p(lat), p(pop)))
    assert nf >= 0
    a = dict(face=np.zeros((nf, 8), np.int32), leaf2=np.zeros((nf, 2), np.int32),
             nodes=np.zeros((nf, 16), np.int32), h=np.zeros(nf), G=np.zeros((nf, 16, 16)))
    shim().shim_ghost_arrays(p(a["face"]), p(a["leaf2"]), p(a["nodes"]), p(a["h"]), p(a["G"]))
    a["cells"] = t["nodes"]
    return a


@pytest.mark.parametrize("kind,jit", [("c0", None), ("sphere", None), ("sphere", 0), ("cone", 1), ("box", 2)])
def test_host_ghost_faces_and_matrices(kind, jit):
    w, o, st = _case(kind, jit)
    nn = o.counts()["n_node"]
    u = np.random.default_rng(3).normal(size=3 * nn)
    g = o.ghost(st, u)
    pop = g["beta"] > 0.0  # every point has E > 0: a leaf is populated iff its maximum is positive
    a = _host_ghost(w, o, pop)
    assert np.array_equal(a["face"], o.ghost_faces())
    assert np.array_equal(a["leaf2"], a["face"][:, :2])
    if kind == "c0":
        assert a["face"].shape[0] == 176
    # same node sets: the union of the two leaves' slot nodes
    lib_cells = a["cells"]
    for i in range(a["face"].shape[0]):
        ids = a["nodes"][i]
        union = set(lib_cells[a["leaf2"][i, 0]]) | set(lib_cells[a["leaf2"][i, 1]])
        assert set(ids[ids >= 0]) == union and np.all(ids[len(union):] == -1)
    G = a["G"]
    assert np.array_equal(G, G.transpose(0, 2, 1)) or np.abs(G - G.transpose(0, 2, 1)).max() <= 1e-15 * np.abs(G).max()
    # penalty as a quadratic form: library matrices against the oracle's assembled K_G
    U = u.reshape(-1, 3)
    val = 0.0
    for i in range(a["face"].shape[0]):
        ids = a["nodes"][i]
        k = ids >= 0
        sc = a["h"][i] * max(g["beta"][a["leaf2"][i, 0]], g["beta"][a["leaf2"][i, 1]])
        Ui = U[ids[k]]
        val += sc * np.sum(G[i][np.ix_(k, k)] * (Ui @ Ui.T))
    rp, col = o.csr()
    Kg = sp.csr_matrix((g["K"], col, rp), shape=(3 * nn, 3 * nn))
    ref = u @ (Kg @ u)
    assert abs(val - ref) <= 1e-12 * abs(ref)
    # h_F / kappa: the larger side of the two leaves over 10
    lv = o.leaves()
    side = w.h_min * np.left_shift(1, w.lvl_max - lv[:, 3]).astype(np.float64)
    hF = np.maximum(side[a["leaf2"][:, 0]], side[a["leaf2"][:, 1]])
    assert np.allclose(a["h"], hF / 10.0, rtol=1e-15, atol=0)


def test_host_ghost_no_faces_without_empty_neighbours():
    w = tiny_workload("sphere", E=1e4)
    o = OracleMesh(w.crit())
    n_leaf = o.leaves().shape[0]
    assert _host_ghost(w, o, np.ones(n_leaf, bool))["face"].shape[0] == 0
    assert _host_ghost(w, o, np.zeros(n_leaf, bool))["face"].shape[0] == 0
