"""Pins of the oracle's octree, hanging-node constraints, numbering, point order and CSR.

Each check uses an independent route: closed-form counts, brute force over all
(node, leaf) / (leaf, leaf) pairs in numpy, linear reproduction of the constraints,
or a different construction of the same set.
"""
import json
import math
from pathlib import Path

import numpy as np
import pytest

import workloads as W
from oracle.oracle import OracleMesh
from tests.helpers import leaf_sizes, morton3_np, node_xyz, setup, tiny_workload

GOLD = Path(__file__).resolve().parent / "golden"
TINY = ["sphere", "cone", "box"]


def test_c0_closed_form_counts():
    g = json.loads((GOLD / "c0_counts.json").read_text())
    w = W.get("c0")
    m, ps = setup(w)
    c = m.counts()
    rp, col = m.csr()
    assert c["n_leaf"] == g["n_leaf"] and c["n_node"] == g["n_node"] and c["n_hang"] == 0
    assert ps.n == g["n_point"]
    assert c["nnz"] == g["nnz"]
    empty = int(np.sum(np.diff(rp) == 0))
    assert empty == g["empty_rows"]
    assert (3 * c["n_node"] - empty) // 3 == g["n_active_nodes"]


def _face_edge_adjacent(w, lv):
    """Pairs of leaves whose closed boxes share a face patch or an edge segment (all pairs)."""
    s = leaf_sizes(w, lv)
    lo = lv[:, :3].astype(np.int64)
    hi = lo + s[:, None]
    ov = np.minimum(hi[:, None, :], hi[None, :, :]) - np.maximum(lo[:, None, :], lo[None, :, :])
    touch = np.all(ov >= 0, axis=2)
    npos = np.sum(ov > 0, axis=2)
    adj = touch & (npos >= 1) & (npos <= 2)
    np.fill_diagonal(adj, False)
    return adj


@pytest.mark.parametrize("kind", TINY)
def test_tiles_domain_and_balance_bruteforce(kind):
    w = tiny_workload(kind, lvl_extra=3)
    m = OracleMesh(w.crit())
    lv = m.leaves()
    s = leaf_sizes(w, lv)
    dims = w.lattice_dims()
    occ = np.zeros(dims[::-1], np.int32)
    for (x, y, z, _), e in zip(lv, s):
        occ[z:z + e, y:y + e, x:x + e] += 1
    assert np.all(occ == 1), "leaves must tile the domain without overlap"
    assert lv[:, 3].max() == w.lvl_max, "the body must trigger refinement to the maximum level"
    adj = _face_edge_adjacent(w, lv)
    i, j = np.nonzero(adj)
    assert np.all(np.abs(lv[i, 3] - lv[j, 3]) <= 1), "2:1 balance across faces and edges"


@pytest.mark.parametrize("kind", ["sphere", "box"])
def test_refinement_criterion_reached(kind):
    """No leaf coarser than the maximum level may meet the body or carry a vertex within
    dx_region of it (Steps 1-3 repeated until nothing is marked)."""
    w = tiny_workload(kind, lvl_extra=3)
    m = OracleMesh(w.crit())
    lv = m.leaves()
    s = leaf_sizes(w, lv)
    b = w.body
    t = np.linspace(0.0, 1.0, 7)
    gz, gy, gx = np.meshgrid(t, t, t, indexing="ij")
    for (x, y, z, lev), e in zip(lv, s):
        if lev == w.lvl_max:
            continue
        lo = np.array([x, y, z]) * w.h_min
        h = e * w.h_min
        P = lo[:, None] + h * np.stack([gx.ravel(), gy.ravel(), gz.ravel()])
        assert not np.any(W.generate._inside_body(w, P[0], P[1], P[2]))
        V = lo[:, None] + h * np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)]).T
        if kind == "sphere":
            d = np.sqrt(((V - np.array(b[:3])[:, None]) ** 2).sum(0)) - b[3]
        else:
            blo, bhi = np.array(b[0::2]), np.array(b[1::2])
            d = np.sqrt((np.maximum(0, np.maximum(blo[:, None] - V, V - bhi[:, None])) ** 2).sum(0))
        assert np.all(d > w.dx_region)


@pytest.mark.parametrize("kind", TINY)
def test_morton_order(kind):
    w = tiny_workload(kind)
    m = OracleMesh(w.crit())
    lv = m.leaves()
    k = morton3_np(lv[:, 0], lv[:, 1], lv[:, 2])
    assert np.all(k[1:] > k[:-1])
    nd = m.nodes()
    kn = morton3_np(nd[:, 0], nd[:, 1], nd[:, 2])
    assert np.all(kn[1:] > kn[:-1])


def _all_nodes(w, lv):
    s = leaf_sizes(w, lv)
    V = []
    for c in range(8):
        o = np.array([c & 1, (c >> 1) & 1, (c >> 2) & 1])
        V.append(lv[:, :3] + o[None, :] * s[:, None])
    V = np.unique(np.concatenate(V), axis=0)
    return V


@pytest.mark.parametrize("kind", TINY)
def test_hanging_set_bruteforce(kind):
    """n hangs iff x_n lies on the boundary of some element K and is not a vertex of K."""
    w = tiny_workload(kind)
    m = OracleMesh(w.crit())
    lv = m.leaves()
    s = leaf_sizes(w, lv)
    V = _all_nodes(w, lv)
    lo = lv[:, :3][None, :, :]
    hi = lo + s[None, :, None]
    P = V[:, None, :]
    inside_closed = np.all((P >= lo) & (P <= hi), axis=2)
    on_face = np.any((P == lo) | (P == hi), axis=2)
    is_vertex = np.all((P == lo) | (P == hi), axis=2)
    hang_on = inside_closed & on_face & ~is_vertex          # (node, leaf)
    hanging = np.any(hang_on, axis=1)
    ijk, sup, wts, own = m.hanging()
    got = {tuple(r) for r in ijk}
    exp = {tuple(r) for r in V[hanging]}
    assert got == exp
    assert m.counts()["n_node"] + m.counts()["n_hang"] == V.shape[0]
    # K_n is the coarsest element the node hangs on
    idx = {tuple(r): i for i, r in enumerate(V)}
    for r, o in zip(ijk, own):
        cand = np.nonzero(hang_on[idx[tuple(r)]])[0]
        assert lv[o, 3] == lv[cand, 3].min()


@pytest.mark.parametrize("name", ["tiny_sphere", "tiny_cone", "c1"])
def test_constraints_reproduce_linear_fields(name):
    """Every hanging node is an edge midpoint (2 supports, 1/2) or a face centre (4, 1/4),
    its supports are independent, and the weights interpolate x exactly."""
    w = W.get(name) if name == "c1" else tiny_workload(name.split("_")[1])
    m = OracleMesh(w.crit())
    ijk, sup, wts, own = m.hanging()
    nodes = m.nodes()
    nsup = np.sum(sup >= 0, axis=1)
    assert set(np.unique(nsup)) <= {2, 4}
    for k in (2, 4):
        sel = nsup == k
        assert np.all(wts[sel][:, :k] == 1.0 / k)
    X = np.zeros(ijk.shape, np.float64)
    for r in range(4):
        ok = sup[:, r] >= 0
        X[ok] += wts[ok, r][:, None] * nodes[sup[ok, r]]
    assert np.array_equal(X, ijk.astype(np.float64))


@pytest.mark.parametrize("name", ["tiny_box", "c1"])
def test_independent_sets_and_modified_basis(name):
    """|I(K)| = 8 under face/edge balance; C_K rows sum to one and map the independent
    nodes' coordinates to each vertex's coordinates (linear reproduction of phi~)."""
    w = W.get(name) if name == "c1" else tiny_workload(name.split("_")[1])
    m = OracleMesh(w.crit())
    n, ids, cm = m.cells()
    assert np.all(n == 8)
    assert np.allclose(cm[:, :, :8].sum(axis=2), 1.0, atol=0, rtol=0)
    lv = m.leaves()
    s = leaf_sizes(w, lv)
    nodes = m.nodes().astype(np.float64)
    X = np.einsum("evz,ezc->evc", cm[:, :, :8], nodes[ids[:, :8]])
    off = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)])
    Xv = lv[:, None, :3] + off[None, :, :] * s[:, None, None]
    assert np.array_equal(X, Xv.astype(np.float64))


@pytest.mark.parametrize("kind,jit", [("sphere", None), ("sphere", 0), ("cone", 1), ("box", 2)])
def test_point_order_and_csr_bruteforce(kind, jit):
    w = tiny_workload(kind)
    m, ps = setup(w, jitter=jit)
    lv = m.leaves()
    # point order: (leaf containing the centre, original index)
    keys = morton3_np(lv[:, 0], lv[:, 1], lv[:, 2])
    q = np.floor((ps.x - np.asarray(w.lo)[:, None]) / w.h_min).astype(np.int64)
    for a, d in enumerate(w.lattice_dims()):
        q[a] = np.clip(q[a], 0, d - 1)
    leaf = np.searchsorted(keys, morton3_np(q[0], q[1], q[2]), side="right") - 1
    order = np.lexsort((np.arange(ps.n), leaf))
    perm, pleaf, nleaf = m.perm()
    assert np.array_equal(pleaf, leaf)
    assert np.array_equal(perm, order)
    if jit is not None:
        assert np.sum(nleaf > 1) > ps.n // 4, "jittered domains must straddle leaves"
    # CSR = node pairs sharing a point's support, 3x3 dense blocks, ascending columns
    pairs = set()
    for p in range(ps.n):
        nd, S, dS = m.point_basis(ps.x[:, p], ps.l[:, p])
        for a in nd:
            for b in nd:
                pairs.add((int(a), int(b)))
    rp, col = m.csr()
    nn = m.counts()["n_node"]
    got = set()
    for a in range(nn):
        for c in range(3):
            cols = col[rp[3 * a + c]:rp[3 * a + c + 1]]
            assert np.all(np.diff(cols) > 0)
            assert np.array_equal(cols % 3, np.tile([0, 1, 2], cols.size // 3))
            if c == 0:
                got |= {(a, int(b) // 3) for b in cols[::3]}
            else:
                assert np.array_equal(cols, col[rp[3 * a]:rp[3 * a + 1]])
    assert got == pairs
