"""GPU parity on meshes whose points all, or all but a few, overlap several leaves.

With every domain over several leaves the fast path has no points at all (no wavefront, no
segment, every node row gathered from the general path alone); with a handful of one-leaf
points it runs over a list shorter than one wavefront while the rest run beside it on the
mesh's second stream. Points are centred on the interior vertices of the leaves of a tiny mesh
with hanging nodes (half-side h_min / 4, so each domain overlaps every leaf touching its
vertex: 2 to 8 of them), plus optionally the centres of a few leaves (half-side a quarter of
the leaf). The library's results are compared with the FP64 oracle on the same points and
seeded state: assembly (f_int, K, sigma, residual and its norm, committed history), dynamic
assembly, body force and adjoint, in FP64 within 1e-11 and with the FP32 tangent within the
bounds of the other parity tests.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.oracle import OracleMesh, residual
from tests.gpu_common import log, rel_err, to_np
from tests.helpers import tiny_workload
from workloads.generate import PointSet

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 2e-5
DT = 2e-3


def _points(w, lv, n_centres):
    hmin = w.h_min
    lo = np.asarray(w.lo, np.float64)
    top = lo + np.asarray(w.base, np.float64) * w.h0
    corner = lv[:, :3].astype(np.float64) * hmin + lo
    inner = np.all((corner > lo + 1e-12) & (corner < top - 1e-12), axis=1)
    v = np.unique(corner[inner], axis=0).T
    x, l = [v], [np.full(v.shape, hmin / 4)]
    if n_centres:
        size = (1 << (w.lvl_max - lv[:n_centres, 3])).astype(np.float64) * hmin
        x.append((corner[:n_centres] + size[:, None] / 2).T)
        l.append(np.tile(size / 4, (3, 1)))
    return PointSet(np.ascontiguousarray(np.concatenate(x, axis=1)), np.ascontiguousarray(np.concatenate(l, axis=1)))


def _setup(n_centres):
    from paper_2606_09275_amd.mesh import Mesh
    w = tiny_workload("sphere", E=1e4, nu=0.3, sy=40.0, Fn_std=0.03)
    o = OracleMesh(w.crit())
    ps = _points(w, o.leaves(), n_centres)
    o.set_points(ps.x, ps.l)
    m = Mesh(w.crit(), torch.from_numpy(ps.x).cuda(), torch.from_numpy(ps.l).cuda())
    log(f"[setup] straddle edges: {ps.n} points, {n_centres} in one leaf, straddle={m.info['n_straddle']}")
    assert m.info["n_straddle"] == ps.n - n_centres
    nodes = o.nodes()
    st = W.make_state(w, ps)
    u = W.make_u(w, nodes, amp=2e-3)
    return w, o, m, ps, st, u, nodes


CASES = [0, 5]


@pytest.mark.parametrize("n_centres", CASES)
def test_assembly_commit_and_body_force(n_centres):
    w, o, m, ps, st, u, nodes = _setup(n_centres)
    ref = o.assemble(st, u)
    fe_ref = o.external_force(dict(st, g=(0.0, 0.0, -9.81)))
    d = W.dirichlet_dofs(nodes)
    r_ref, rn_ref = residual(ref["f_int"], fe_ref, d)
    perm = to_np(m.arrays()["perm"])
    s_dev = m.sorted_state(dict(st, g=(0.0, 0.0, -9.81)))
    ud, dd = torch.from_numpy(u).cuda(), torch.from_numpy(d).cuda()
    fe = m.external_force(s_dev)
    out = m.assemble(s_dev, ud, "f64", f_ext=fe, dirichlet=dd, commit=True)
    torch.cuda.synchronize()
    e = {"f": rel_err(to_np(out["f_int"]), ref["f_int"]), "K": rel_err(to_np(out["K"]), ref["K"]),
         "sigma": rel_err(to_np(out["sigma"]), ref["sigma"][:, perm]),
         "F_new": rel_err(to_np(out["F_new"]), ref["Fnew"][:, perm]),
         "b_e": rel_err(to_np(out["be_new"]), ref["be"][:, perm]),
         "fext": rel_err(to_np(fe), fe_ref), "r": rel_err(to_np(out["r"]), r_ref),
         "rnorm": abs(float(to_np(out["rnorm"])[0]) - rn_ref) / rn_ref}
    log(f"[parity] straddle edges {n_centres} fp64 plastic={ref['plastic'].mean():.2f} " +
        " ".join(f"{k}={v:.2e}" for k, v in e.items()))
    assert all(v <= TOL64 for v in e.values()), e
    o32 = m.assemble(s_dev, ud, "f32k", f_ext=fe, dirichlet=dd)
    torch.cuda.synchronize()
    e32 = {"f": rel_err(to_np(o32["f_int"]), ref["f_int"]), "K": rel_err(to_np(o32["K"]), ref["K"]),
           "r": rel_err(to_np(o32["r"]), r_ref), "rnorm": abs(float(to_np(o32["rnorm"])[0]) - rn_ref) / rn_ref}
    log(f"[parity] straddle edges {n_centres} fp32k " + " ".join(f"{k}={v:.2e}" for k, v in e32.items()))
    assert all(v <= TOL32 for v in e32.values()), e32


@pytest.mark.parametrize("n_centres", CASES)
def test_dynamic_assembly(n_centres):
    w, o, m, ps, st, u, nodes = _setup(n_centres)
    vel = W.make_velocity(w, ps)
    ref = o.assemble(st, u)
    ine = o.inertia(st, u, vel, DT)
    perm = to_np(m.arrays()["perm"])
    s_dev = m.sorted_state(st)
    v_dev = torch.from_numpy(np.ascontiguousarray(vel[:, perm])).cuda()
    out = m.assemble_dynamic(s_dev, torch.from_numpy(u).cuda(), v_dev, DT, "f64", want_kinematics=True)
    torch.cuda.synchronize()
    e = {"f": rel_err(to_np(out["f_int"]), ref["f_int"] + ine["f_iner"]),
         "K": rel_err(to_np(out["K"]), ref["K"] + ine["K_mass"]),
         "a": rel_err(to_np(out["a_new"]), ine["a"][:, perm]), "v": rel_err(to_np(out["v_new"]), ine["v"][:, perm])}
    log(f"[parity] straddle edges {n_centres} dynamic " + " ".join(f"{k}={v:.2e}" for k, v in e.items()))
    assert all(v <= TOL64 for v in e.values()), e


@pytest.mark.parametrize("n_centres", CASES)
def test_adjoint(n_centres):
    w, o, m, ps, st, u, nodes = _setup(n_centres)
    lam = W.make_lambda(w, nodes)
    ref = o.adjoint(st, u, lam)
    perm = to_np(m.arrays()["perm"])
    s_dev = m.sorted_state(st)
    ud, ld = torch.from_numpy(u).cuda(), torch.from_numpy(lam).cuda()
    for prec, tol in (("f64", TOL64), ("f32k", 2e-4)):
        g = m.adjoint(s_dev, ud, ld, prec)
        torch.cuda.synchronize()
        errs = {k: rel_err(to_np(g[k]), ref[k][perm]) for k in ("dE", "dnu", "dsy", "dV")}
        log(f"[parity] straddle edges {n_centres} adjoint {prec} " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
        assert all(v <= tol for v in errs.values()), errs
