"""Pins of the oracle's GIMP refinement (Section 5): the paper's one-dimensional worked example,
children that tile the parent domain, conservation of volume, mass and first moment, the
reference-position map (x_c - x = F_n (X_c - X)), copies of unsplit points and of constant
data, and the criterion l_K < beta l_p on meshes with known leaf sizes."""
import json
from pathlib import Path

import numpy as np
import pytest

import workloads as W
from oracle.oracle import OracleMesh
from oracle.split import split_points
from tests.helpers import tiny_workload

GOLDEN = Path(__file__).resolve().parent / "golden" / "split_1d_example.json"


def _state(x, l, Fn, rng):
    n = x.shape[1]
    F = Fn.reshape(3, 3, n)
    b = np.einsum("ijn,kjn->ikn", F, F)
    return dict(x=x, l=l, vol=8 * l.prod(axis=0), mass=2.0 * 8 * l.prod(axis=0),
                Jn=np.linalg.det(F.transpose(2, 0, 1)),
                bn=np.stack([b[0, 0], b[1, 1], b[2, 2], b[0, 1], b[1, 2], b[0, 2]]),
                Fn=Fn, E=rng.uniform(1e3, 2e3, n), nu=np.full(n, 0.3), sy=rng.uniform(5, 10, n))


def test_paper_one_dimensional_example():
    g = json.loads(GOLDEN.read_text())
    zc, Lc = g["parent_current"]["z"], g["parent_current"]["length"]
    zr, Lr = g["parent_reference"]["z"], g["parent_reference"]["length"]
    stretch = Lc / Lr
    x = np.array([[0.5], [0.5], [zc]])
    l = np.array([[0.05], [0.05], [Lc / 2]])
    Fn = np.diag([1.0, 1.0, stretch]).reshape(9, 1)
    s = _state(x, l, Fn, np.random.default_rng(0))
    X = np.array([[0.5], [0.5], [zr]])
    out = split_points(s, np.array([1], np.uint8), X=X, props={"E": (1.0, 0.0, 0.0, -1.0)})
    z = out["x"][2]
    assert sorted(set(np.round(z, 12))) == g["children_current"]["z"]
    assert np.allclose(2 * out["l"][2], g["children_current"]["length"], rtol=0, atol=1e-15)
    Z = out["X"][2]
    assert sorted(set(np.round(Z, 12))) == g["children_reference"]["z"]
    # E = 1 - Z at the children's own reference positions, not the parent's 0.75
    assert np.allclose(out["E"], 1.0 - Z, rtol=0, atol=1e-15)
    assert sorted(set(np.round(out["E"], 12))) == [0.625, 0.875]


def _random_points(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.2, 0.8, (3, n))
    l = rng.uniform(0.01, 0.05, (3, n))
    Fn = (np.eye(3)[:, :, None] + rng.normal(0, 0.1, (3, 3, n))).reshape(9, n)
    return x, l, Fn, rng


def test_children_tile_the_parent_and_conserve():
    x, l, Fn, rng = _random_points(20, 1)
    s = _state(x, l, Fn, rng)
    split = np.ones(20, np.uint8)
    X = x + rng.normal(0, 0.01, x.shape)
    v = rng.normal(size=(3, 20))
    out = split_points(s, split, X=X, v=v)
    assert out["x"].shape == (3, 160)
    for p in range(20):
        ch = slice(8 * p, 8 * p + 8)
        lo = out["x"][:, ch] - out["l"][:, ch]
        hi = out["x"][:, ch] + out["l"][:, ch]
        assert np.allclose(lo.min(axis=1), x[:, p] - l[:, p], rtol=0, atol=1e-15)
        assert np.allclose(hi.max(axis=1), x[:, p] + l[:, p], rtol=0, atol=1e-15)
        # disjoint boxes filling the parent: volumes add up and every pair is separated on an axis
        assert np.isclose(np.prod(hi - lo, axis=0).sum(), np.prod(2 * l[:, p]), rtol=1e-13)
        for i in range(8):
            for j in range(i + 1, 8):
                sep = (hi[:, i] <= lo[:, j] + 1e-15) | (hi[:, j] <= lo[:, i] + 1e-15)
                assert sep.any()
        assert out["vol"][ch].sum() == s["vol"][p] and out["mass"][ch].sum() == s["mass"][p]
        mom = (out["mass"][ch] * out["x"][:, ch]).sum(axis=1)
        assert np.allclose(mom, s["mass"][p] * x[:, p], rtol=1e-15, atol=0)
        # reference map: x_c - x = F (X_c - X); the children's reference centres average to X
        F = Fn[:, p].reshape(3, 3)
        d = F @ (out["X"][:, ch] - X[:, [p]])
        assert np.allclose(d, out["x"][:, ch] - x[:, [p]], rtol=0, atol=1e-14)
        assert np.allclose(out["X"][:, ch].mean(axis=1), X[:, p], rtol=0, atol=1e-15)
        # constant data copied
        for k in ("Jn", "E", "nu", "sy"):
            assert np.all(out[k][ch] == s[k][p])
        for k in ("bn", "Fn"):
            assert np.all(out[k][:, ch] == s[k][:, [p]])
        assert np.all(out["v"][:, ch] == v[:, [p]])


def test_unsplit_points_are_copied_in_order():
    x, l, Fn, rng = _random_points(10, 2)
    s = _state(x, l, Fn, rng)
    split = np.array([0, 1, 0, 0, 1, 0, 0, 0, 1, 0], np.uint8)
    out = split_points(s, split)
    assert out["x"].shape[1] == 10 + 7 * 3
    src = np.repeat(np.arange(10), np.where(split == 1, 8, 1))
    keep = np.repeat(split == 0, np.where(split == 1, 8, 1))
    for k in s:
        a = np.asarray(s[k]).reshape(-1, 10)
        b = np.asarray(out[k]).reshape(-1, out["x"].shape[1])
        assert np.array_equal(b[:, keep], a[:, src[keep]])
    # children of the second point sit in child order: bit a of c set <=> offset +l_a / 2
    ch = out["x"][:, 1:9] - x[:, [1]]
    for c in range(8):
        assert all((ch[a, c] > 0) == bool((c >> a) & 1) for a in range(3))


def test_criterion_on_a_uniform_mesh():
    """Unrefined mesh (3^3 base cells of side h): points two per axis per leaf have l_p = h/4 and
    l_K = h/2 = 2 l_p, so beta = 2 splits none and any beta > 2 splits all; points four per axis
    (l_p = h/8) stay unsplit for beta up to 4."""
    w = tiny_workload("none")
    o = OracleMesh(w.crit())
    lv = o.leaves()
    h = w.h_min * (1 << (w.lvl_max - lv[0, 3]))
    assert np.all(lv[:, 3] == lv[0, 3])
    ps = W.make_points(w, lv[:, :3], lv[:, 3])
    assert np.allclose(ps.l, h / 4)
    assert o.split_mark(ps.x, ps.l, 2.0).sum() == 0
    assert o.split_mark(ps.x, ps.l, 2.0 + 1e-9).all()
    w.ppa = lambda lev: 4
    ps4 = W.make_points(w, lv[:, :3], lv[:, 3])
    assert o.split_mark(ps4.x, ps4.l, 4.0).sum() == 0
    assert o.split_mark(ps4.x, ps4.l, 4.0 + 1e-9).all()


@pytest.mark.parametrize("kind", ["sphere", "cone", "box"])
def test_criterion_on_a_refined_mesh(kind):
    """Points laid out for the base level (two per axis per base cell) on the refined mesh: a
    point is split iff some finest-lattice cell under its domain belongs to a leaf finer than
    the base level (l_K <= h_base / 4 < 2 l_p); the largest half side decides."""
    w = tiny_workload(kind)
    o = OracleMesh(w.crit())
    lv = o.leaves()
    base = np.array([[i, j, k] for k in range(w.base[2]) for j in range(w.base[1]) for i in range(w.base[0])])
    s0 = 1 << (w.lvl_max - w.lvl_base)
    ps = W.make_points(w, base * s0, np.full(base.shape[0], w.lvl_base))
    flags = o.split_mark(ps.x, ps.l, 2.0)
    # brute force over the finest cells under each domain
    lat = np.array(w.lattice_dims())
    cell_level = np.zeros(tuple(lat), np.int32)
    for q in lv:
        s = 1 << (w.lvl_max - q[3])
        cell_level[q[0]:q[0] + s, q[1]:q[1] + s, q[2]:q[2] + s] = q[3]
    ref = np.zeros(ps.n, np.uint8)
    for p in range(ps.n):
        lo = np.floor((ps.x[:, p] - ps.l[:, p]) / w.h_min + 1e-9).astype(int)
        hi = np.ceil((ps.x[:, p] + ps.l[:, p]) / w.h_min - 1e-9).astype(int)
        ref[p] = cell_level[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].max() > w.lvl_base
    assert np.array_equal(flags, ref) and 0 < flags.sum() < ps.n
    # anisotropic domain: the largest half side decides
    l2 = ps.l.copy()
    l2[0] *= 0.5
    l2[1] *= 0.5
    assert np.array_equal(o.split_mark(ps.x, l2, 2.0), ref)


def test_repeated_split_until_the_criterion_holds():
    """Base-level points on a mesh refined two levels: children overlapping the finest leaves
    are split again; after the rounds no point meets the criterion and the volume is kept."""
    w = tiny_workload("sphere", lvl_extra=2)
    o = OracleMesh(w.crit())
    base = np.array([[i, j, k] for k in range(w.base[2]) for j in range(w.base[1]) for i in range(w.base[0])])
    s0 = 1 << (w.lvl_max - w.lvl_base)
    ps = W.make_points(w, base * s0, np.full(base.shape[0], w.lvl_base))
    rng = np.random.default_rng(5)
    Fn = np.tile(np.eye(3).reshape(9, 1), ps.n)
    s = _state(ps.x, ps.l, Fn, rng)
    vol0 = s["vol"].sum()
    rounds = 0
    while True:
        f = o.split_mark(s["x"], s["l"], 2.0)
        if not f.any():
            break
        s = split_points(s, f)
        rounds += 1
    assert rounds == 2
    assert np.isclose(s["vol"].sum(), vol0, rtol=1e-14)
