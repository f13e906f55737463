"""GPU parity of the GIMP refinement (Section 5) through the C ABI against the oracle: the split
flags bit-exact on meshes with hanging nodes (lattice and jittered points, anisotropic domains,
the full-size cone-penetration mesh), the split points (positions, half sides, volumes,
masses and copied data bit-exact; reference positions and reference-position parameters
within 1e-13), the paper's one-dimensional example, repeated rounds, and argument errors."""
import dataclasses
import json
import math
from pathlib import Path

import numpy as np
import pytest
import torch

import workloads as W
from oracle.oracle import OracleMesh
from oracle.split import split_points
from tests.gpu_common import log, rel_err, to_np
from tests.helpers import tiny_workload

pytestmark = pytest.mark.gpu

GOLDEN = Path(__file__).resolve().parent / "golden" / "split_1d_example.json"
FIELDS = {"x": 3, "l": 3, "vol": 1, "mass": 1, "Jn": 1, "bn": 6, "Fn": 9, "E": 1, "nu": 1, "sy": 1}


def _base_points(w, jit=None):
    """Points laid out for the base level (2 per axis per base cell) of w's mesh."""
    base = np.array([[i, j, k] for k in range(w.base[2]) for j in range(w.base[1]) for i in range(w.base[0])])
    s0 = 1 << (w.lvl_max - w.lvl_base)
    ps = W.make_points(w, base * s0, np.full(base.shape[0], w.lvl_base))
    if jit is not None:
        ps = W.jitter_points(w, ps, jit)
    return ps


def _state(ps, seed):
    rng = np.random.default_rng(seed)
    n = ps.n
    F = np.eye(3)[:, :, None] + rng.normal(0, 0.05, (3, 3, n))
    b = np.einsum("ijn,kjn->ikn", F, F)
    return dict(x=ps.x, l=ps.l, vol=8 * ps.l.prod(axis=0), mass=1.5 * 8 * ps.l.prod(axis=0),
                Jn=np.linalg.det(F.transpose(2, 0, 1)),
                bn=np.stack([b[0, 0], b[1, 1], b[2, 2], b[0, 1], b[1, 2], b[0, 2]]), Fn=F.reshape(9, n),
                E=rng.uniform(1e3, 2e3, n), nu=np.full(n, 0.3), sy=rng.uniform(5.0, 10.0, n))


def _dev(s):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in s.items()}


@pytest.mark.parametrize("kind,jit", [("sphere", None), ("cone", 1), ("box", 2), ("sphere", 0)])
def test_split_flags_match_oracle(kind, jit):
    from paper_2606_09275_amd.mesh import Mesh
    w = tiny_workload(kind)
    o = OracleMesh(w.crit())
    m = Mesh(w.crit())
    ps = _base_points(w, jit)
    ref = o.split_mark(ps.x, ps.l, 2.0)
    flags, cnt = m.split_mark(torch.from_numpy(ps.x).cuda(), torch.from_numpy(ps.l).cuda(), 2.0)
    log(f"[parity] split flags {kind} jit={jit}: {cnt} of {ps.n} (oracle {int(ref.sum())})")
    assert np.array_equal(to_np(flags), ref) and cnt == int(ref.sum()) and 0 < cnt < ps.n
    # anisotropic domains (largest half side decides) and another beta
    l2 = ps.l.copy()
    l2[1] *= 0.5
    for beta in (2.0, 3.0, 4.5):
        f2, c2 = m.split_mark(torch.from_numpy(ps.x).cuda(), torch.from_numpy(l2).cuda(), beta)
        assert np.array_equal(to_np(f2), o.split_mark(ps.x, l2, beta))


@pytest.mark.parametrize("kind,jit", [("sphere", None), ("cone", 1)])
def test_split_apply_matches_oracle(kind, jit):
    from paper_2606_09275_amd.mesh import Mesh
    w = tiny_workload(kind)
    o = OracleMesh(w.crit())
    m = Mesh(w.crit())
    ps = _base_points(w, jit)
    s = _state(ps, 3)
    rng = np.random.default_rng(4)
    X = ps.x + rng.normal(0, 0.01, ps.x.shape)
    v = rng.normal(size=(3, ps.n))
    props = {"E": (1e3, 10.0, -20.0, 30.0), "sy": (7.0, 0.0, 0.0, -1.0)}
    flags = o.split_mark(ps.x, ps.l, 2.0)
    ref = split_points(s, flags, X=X, v=v, props=props)
    sd = _dev(s)
    fl, cnt = m.split_mark(sd["x"], sd["l"], 2.0)
    out = m.split_apply(sd, fl, cnt, X=torch.from_numpy(X).cuda(), v=torch.from_numpy(v).cuda(), props=props)
    torch.cuda.synchronize()
    n_out = ps.n + 7 * cnt
    log(f"[parity] split apply {kind}: {ps.n} -> {n_out} points")
    assert out["x"].shape[1] == n_out == ref["x"].shape[1]
    for k in ("x", "l", "vol", "mass", "Jn", "bn", "Fn", "nu", "v"):
        assert np.array_equal(to_np(out[k]), ref[k]), k
    for k in ("X", "E", "sy"):
        e = rel_err(to_np(out[k]), ref[k])
        log(f"[parity] split {kind} {k}: {e:.2e}")
        assert e <= 1e-13, k


def test_split_paper_one_dimensional_example():
    from paper_2606_09275_amd.mesh import Mesh
    g = json.loads(GOLDEN.read_text())
    w = tiny_workload("none")
    m = Mesh(w.crit())
    zc, Lc = g["parent_current"]["z"], g["parent_current"]["length"]
    zr, Lr = g["parent_reference"]["z"], g["parent_reference"]["length"]
    x = np.array([[0.5], [0.5], [zc]])
    l = np.array([[0.05], [0.05], [Lc / 2]])
    s = dict(x=x, l=l, vol=8 * l.prod(axis=0), mass=8 * l.prod(axis=0), Fn=np.diag([1.0, 1.0, Lc / Lr]).reshape(9, 1),
             E=np.array([1.0 - zr]))
    sd = _dev(s)
    out = m.split_apply(sd, torch.ones(1, dtype=torch.uint8, device="cuda"), 1,
                        X=torch.tensor([[0.5], [0.5], [zr]], dtype=torch.float64, device="cuda"),
                        props={"E": (1.0, 0.0, 0.0, -1.0)})
    z = to_np(out["x"])[2]
    Z = to_np(out["X"])[2]
    assert sorted(set(np.round(z, 12))) == g["children_current"]["z"]
    assert sorted(set(np.round(Z, 12))) == g["children_reference"]["z"]
    assert np.allclose(2 * to_np(out["l"])[2], g["children_current"]["length"], rtol=0, atol=1e-15)
    assert sorted(set(np.round(to_np(out["E"]), 12))) == [0.625, 0.875]


def test_split_rounds_until_the_criterion_holds():
    """Base-level points on a mesh two levels finer near the body: two rounds on the GPU give
    the oracle's points after its two rounds."""
    from paper_2606_09275_amd.mesh import Mesh
    w = tiny_workload("sphere", lvl_extra=2)
    o = OracleMesh(w.crit())
    m = Mesh(w.crit())
    ps = _base_points(w)
    s = _state(ps, 5)
    sd = _dev(s)
    rounds = 0
    while True:
        ref_flags = o.split_mark(s["x"], s["l"], 2.0)
        fl, cnt = m.split_mark(sd["x"], sd["l"], 2.0)
        assert np.array_equal(to_np(fl), ref_flags)
        if cnt == 0:
            break
        s = split_points(s, ref_flags)
        sd = m.split_apply(sd, fl, cnt)
        rounds += 1
        for k in FIELDS:
            assert np.array_equal(to_np(sd[k]), s[k]), k
    assert rounds == 2


def test_split_full_size_cone_mesh():
    """The cone-penetration mesh: its own points (the discretisation the workload uses) are not
    split; points laid out one level coarser are split where the mesh is finest, flags
    bit-exact against the oracle and the split volume conserved."""
    from paper_2606_09275_amd.mesh import Mesh
    w = W.get("c2")
    o = OracleMesh(w.crit())
    m = Mesh(w.crit())
    lv = o.leaves()
    ps = W.make_points(w, lv[:, :3], lv[:, 3])
    fl, cnt = m.split_mark(torch.from_numpy(ps.x).cuda(), torch.from_numpy(ps.l).cuda(), 2.0)
    log(f"[parity] split c2 points: {cnt} of {ps.n}")
    assert cnt == 0
    # one level coarser: 2 points per axis in the parents of the leaves (a domain then overlaps
    # up to 8^3 finest leaves), mixed with every 7th point of the workload's own
    par = lv.copy()
    s = np.left_shift(1, w.lvl_max - (lv[:, 3] - 1))
    par[:, :3] = (lv[:, :3] // s[:, None]) * s[:, None]
    par[:, 3] = lv[:, 3] - 1
    par = np.unique(par[par[:, 3] >= w.lvl_base], axis=0)  # parents that exist in a tree of this base grid
    pc = W.make_points(dataclasses.replace(w, ppa=lambda lev: 2), par[:, :3], par[:, 3])
    x = np.ascontiguousarray(np.concatenate([pc.x, ps.x[:, ::7]], axis=1))
    l = np.ascontiguousarray(np.concatenate([pc.l, ps.l[:, ::7]], axis=1))
    ref = o.split_mark(x, l, 2.0)
    xd, ld = torch.from_numpy(x).cuda(), torch.from_numpy(l).cuda()
    fl, cnt = m.split_mark(xd, ld, 2.0)
    log(f"[parity] split c2 mixed points: {cnt} of {x.shape[1]} (oracle {int(ref.sum())})")
    assert np.array_equal(to_np(fl), ref) and 0 < cnt < x.shape[1]
    vol = torch.from_numpy(8 * l.prod(axis=0)).cuda()
    st = dict(x=xd, l=ld, vol=vol, mass=vol.clone())
    out = m.split_apply(st, fl, cnt)
    assert out["x"].shape[1] == x.shape[1] + 7 * cnt
    assert math.isclose(float(out["vol"].sum()), float(vol.sum()), rel_tol=1e-12)


def test_split_argument_errors():
    from paper_2606_09275_amd._lib import MPMError
    from paper_2606_09275_amd.mesh import Mesh
    w = tiny_workload("sphere")
    m = Mesh(w.crit())
    ps = _base_points(w)
    sd = _dev(_state(ps, 6))
    fl, cnt = m.split_mark(sd["x"], sd["l"], 2.0)
    with pytest.raises(MPMError) as e:  # wrong output count
        m.split_apply(sd, fl, cnt + 1)
    assert e.value.code == -1
    with pytest.raises(MPMError) as e:  # reference-position parameters without X
        m.split_apply(sd, fl, cnt, props={"E": (1.0, 0.0, 0.0, 0.0)})
    assert e.value.code == -1
    with pytest.raises(MPMError) as e:
        m.split_mark(sd["x"], sd["l"], float("nan"))
    assert e.value.code == -1
    x_out = sd["x"].clone()
    x_out[0, 5] = 50.0  # far outside the mesh box
    with pytest.raises(MPMError) as e:
        m.split_mark(x_out, sd["l"], 2.0)
    assert e.value.code == -4 and e.value.index == 5
    l_bad = sd["l"].clone()
    l_bad[1, 7] = float("inf")
    with pytest.raises(MPMError) as e:
        m.split_mark(sd["x"], l_bad, 2.0)
    assert e.value.code == -7 and e.value.index == 7
