"""Pins of the oracle's ghost stabilisation (Section 4): the face set of the uniform mesh in
closed form, zero penalty on displacement fields that are affine (no gradient jump,
including across hanging faces), the exact penalty of a kinked field, symmetry, positive
semi-definiteness, equal-component coupling, the scaling with the Young's modulus and the
per-leaf modulus maximum."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle.oracle import OracleMesh
from tests.helpers import node_xyz, tiny_workload


def _partly_filled(kind):
    """Tiny mesh with hanging nodes whose points fill only the region z < 0.55, so that
    unpopulated leaves border populated ones."""
    w = tiny_workload(kind, E=1e4)
    w.keep = lambda x, y, z: z < 0.55
    return w


def _setup(w, jitter=None, E=None):
    m = OracleMesh(w.crit(), ghost=True)
    lv = m.leaves()
    ps = W.make_points(w, lv[:, :3], lv[:, 3])
    if jitter is not None:
        ps = W.jitter_points(w, ps, jitter)
    m.set_points(ps.x, ps.l)
    s = W.make_state(w, ps)
    if E is not None:
        s["E"] = E(ps)
    return m, ps, s


def _K(m, K):
    rp, col = m.csr()
    n = 3 * m.counts()["n_node"]
    return sp.csr_matrix((K, col, rp), shape=(n, n))


def test_uniform_mesh_faces_closed_form():
    """C0: points fill the lower half (layers 0-3 of 8); layer 3 borders the empty layer 4, so
    its 64 leaves are the boundary leaves; their faces with populated leaves are 64 below and
    2 x 7 x 8 within the layer: 176 ghost faces."""
    m, ps, s = _setup(W.get("c0"))
    f = m.ghost_faces()
    assert f.shape[0] == 176
    lv = m.leaves()
    axis_count = np.bincount(f[:, 2], minlength=3)
    assert axis_count.tolist() == [56, 56, 64]
    # every face touches a layer-3 leaf (z anchor 3 in level-3 units = 3 * 1 lattice cells)
    assert np.all((lv[f[:, 0], 2] == 3) | (lv[f[:, 1], 2] == 3))


def test_kinked_field_penalty_closed_form():
    """u_x = max(0, x - 1/2) jumps in normal derivative by 1 across the plane x = 1/2 only; the
    ghost faces on that plane are the 8 faces of layer 3: u.K_G.u = (h E / 10) * 8 h^2."""
    w = W.get("c0")
    m, ps, s = _setup(w)
    xyz = node_xyz(w, m.nodes())
    u = np.zeros(3 * xyz.shape[0])
    u[0::3] = np.maximum(0.0, xyz[:, 0] - 0.5)
    out = m.ghost(s, u)
    h, E = 0.125, w.E
    val = u @ (_K(m, out["K"]) @ u)
    assert abs(val - (h * E / 10.0) * 8 * h * h) <= 1e-12 * val
    assert abs(u @ out["f"] - val) <= 1e-12 * val


@pytest.mark.parametrize("kind,jit", [("sphere", None), ("cone", 1), ("box", 2)])
def test_affine_fields_have_no_penalty(kind, jit):
    w = _partly_filled(kind)
    m, ps, s = _setup(w, jitter=jit)
    assert m.ghost_faces().shape[0] > 0
    xyz = node_xyz(w, m.nodes())
    rng = np.random.default_rng(9)
    A = rng.normal(size=(3, 3))
    c = rng.normal(size=3)
    u = (xyz @ A.T + c).reshape(-1)
    out = m.ghost(s, u)
    Kg = _K(m, out["K"])
    scale = abs(Kg).max() * np.abs(u).max()
    assert np.abs(out["f"]).max() <= 1e-11 * scale
    assert np.abs(Kg @ u).max() <= 1e-11 * scale


@pytest.mark.parametrize("kind,jit", [("sphere", None), ("cone", 1), ("box", 2)])
def test_symmetric_psd_and_modulus_scaling(kind, jit):
    w = _partly_filled(kind)
    m, ps, s = _setup(w, jitter=jit)
    n_node = m.counts()["n_node"]
    u = np.random.default_rng(2).normal(size=3 * n_node)
    out = m.ghost(s, u)
    Kg = _K(m, out["K"])
    assert abs(Kg - Kg.T).max() <= 1e-14 * abs(Kg).max()
    rng = np.random.default_rng(3)
    for _ in range(5):
        d = rng.normal(size=3 * n_node)
        assert d @ (Kg @ d) >= -1e-13 * abs(Kg).max() * (d @ d)
    # the force is K_G u, and K_G couples only equal displacement components
    assert np.allclose(Kg @ u, out["f"], rtol=0, atol=1e-12 * np.abs(out["f"]).max())
    coo = Kg.tocoo()
    assert np.all(coo.data[(coo.row % 3) != (coo.col % 3)] == 0.0)
    # the same scalar form on the three components
    assert np.array_equal(Kg[0::3, 0::3].toarray(), Kg[1::3, 1::3].toarray())
    s2 = dict(s, E=2.0 * s["E"])
    out2 = m.ghost(s2, u)
    assert np.allclose(out2["K"], 2.0 * out["K"], rtol=1e-15, atol=0)
    assert np.allclose(out2["beta"], 2.0 * out["beta"], rtol=0, atol=0)


def test_beta_is_maximum_modulus_per_leaf():
    """Points lying in one leaf each: beta of a leaf is the largest E of its points, 0 for a
    leaf without points."""
    w = _partly_filled("sphere")
    m, ps, s = _setup(w, E=lambda ps: 1e3 + 1e3 * ps.x[0])
    out = m.ghost(s, np.zeros(3 * m.counts()["n_node"]))
    perm, pleaf, nleaf = m.perm()
    assert np.all(nleaf == 1)
    ref = np.zeros(m.counts()["n_leaf"])
    np.maximum.at(ref, pleaf, s["E"])
    assert np.array_equal(out["beta"], ref)


@pytest.mark.parametrize("kind", ["sphere", "box"])
def test_kinked_field_across_mixed_level_faces(kind):
    """u_x = max(0, x - 1/3): the plane x = 1/3 bounds base cells, so every leaf lies on one
    side and the field is linear in each leaf; its normal derivative jumps by 1 on every face
    of that plane, whatever the two leaves' sizes: u.K_G.u = sum over the ghost faces of the
    plane of (h_F E / 10) |F|, h_F the larger side of the two leaves."""
    w = _partly_filled(kind)
    m, ps, s = _setup(w)
    xyz = node_xyz(w, m.nodes())
    u = np.zeros(3 * xyz.shape[0])
    u[0::3] = np.maximum(0.0, xyz[:, 0] - 1.0 / 3.0)
    out = m.ghost(s, u)
    val = u @ (_K(m, out["K"]) @ u)
    f = m.ghost_faces()
    lv = m.leaves()
    plane = round((1.0 / 3.0) / w.h_min)
    on = f[(f[:, 2] == 0) & (f[:, 3] == plane)]
    assert on.shape[0] > 0
    sides = w.h_min * np.left_shift(1, w.lvl_max - lv[:, 3]).astype(np.float64)
    hF = np.maximum(sides[on[:, 0]], sides[on[:, 1]])
    area = (on[:, 5] - on[:, 4]) * (on[:, 7] - on[:, 6]) * w.h_min ** 2
    assert np.any(sides[on[:, 0]] != sides[on[:, 1]])  # faces between leaves of two sizes
    ref = np.sum(hF * w.E / 10.0 * area)
    assert abs(val - ref) <= 1e-11 * ref
