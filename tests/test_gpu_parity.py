"""GPU parity: the HIP library through its C ABI against the FP64 oracle on the same seeded
inputs. Integers (leaves, nodes, constraints, point order, CSR) bit-exact; FP64 results
within 1e-11 normwise (max|diff| / max|ref|); FP32-tangent results within stated bounds."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_common import build_pair, log, rel_err, to_np
from tests.helpers import tiny_workload

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
# FP32 tangent path: basis, stress, tangent and K in FP32 (unit roundoff 6e-8); f_int and the
# residual accumulate in FP64. Bounds: a few hundred ulps of the FP32 working precision.
TOL32_F = 2e-5
TOL32_K = 2e-5
TOL32_SIG = 2e-5


def _mesh_checks(o, m, ps):
    a = m.arrays()
    assert np.array_equal(to_np(a["leaf"]), o.leaves())
    assert np.array_equal(to_np(a["node_ijk"]), o.nodes())
    ijk, sup, wt, own = o.hanging()
    assert np.array_equal(to_np(a["hang_ijk"]), ijk)
    assert np.array_equal(to_np(a["hang_owner"]), own)
    perm_o, pleaf_o, nleaf_o = o.perm()
    perm = to_np(a["perm"])
    assert np.array_equal(perm, perm_o)
    assert np.array_equal(to_np(a["point_leaf"]), pleaf_o[perm])
    assert np.array_equal(to_np(a["point_nleaf"]), nleaf_o[perm])
    rp, col = o.csr()
    assert np.array_equal(to_np(a["row_ptr"]), rp)
    assert np.array_equal(to_np(a["col"]), col)
    c = o.counts()
    assert m.info["nnz"] == c["nnz"] and m.info["n_straddle"] == c["n_straddle"]
    assert m.info["n_active_rows"] == c["n_active_rows"]


def _inputs(w, o, ps, m, u_amp=1e-3):
    st = W.make_state(w, ps)
    nodes = o.nodes()
    u = W.make_u(w, nodes, amp=u_amp)
    s_dev = m.sorted_state(dict(st, g=(0.0, 0.0, -9.81)))
    return st, u, s_dev, nodes


CASES = [
    ("c0", None, None),
    ("tiny_sphere_el", "sphere", None),
    ("tiny_sphere_jit", "sphere", 0),
    ("tiny_cone_vm_jit", "cone", 1),
    ("tiny_box_vm", "box", None),
    # coarse leaves holding 12^3 points (27 wavefront segments: one summed record per leaf)
    ("tiny_sphere_heavy_vm", "sphere", None),
    # coarse leaves holding 20^3 points (125 segments: chunk sums, then the leaf sum), jittered
    ("tiny_box_heavy2_jit", "box", 2),
]

_HEAVY_PPA = {"heavy": lambda lv: 12 if lv == 2 else 2, "heavy2": lambda lv: 20 if lv == 2 else 3}


def _work(tag, kind):
    if kind is None:
        return W.get(tag)
    sy = math.inf if tag.endswith("_el") else (5.0 if "vm" in tag else 40.0)
    ppa = 2
    for key in ("heavy2", "heavy"):
        if f"_{key}" in tag:
            ppa = _HEAVY_PPA[key]
            break
    return tiny_workload(kind, E=1e4, nu=0.3, sy=sy, Fn_std=0.03, ppa=ppa)


@pytest.mark.parametrize("tag,kind,jit", CASES)
def test_mesh_order_csr_bitexact(tag, kind, jit):
    w = _work(tag, kind)
    o, m, ps = build_pair(w, jitter=jit)
    _mesh_checks(o, m, ps)


@pytest.mark.parametrize("tag,kind,jit", CASES)
def test_assemble_fp64_matches_oracle(tag, kind, jit):
    w = _work(tag, kind)
    o, m, ps = build_pair(w, jitter=jit)
    st, u, s_dev, nodes = _inputs(w, o, ps, m, u_amp=2e-3)
    ref = o.assemble(st, u)
    fe_ref = o.external_force(dict(st, g=(0.0, 0.0, -9.81)))
    d = W.dirichlet_dofs(nodes)
    from oracle.oracle import residual
    r_ref, rn_ref = residual(ref["f_int"], fe_ref, d)
    log(f"[run] {tag} fp64 assemble n={ps.n} nnz={m.info['nnz']} straddle={m.info['n_straddle']}")
    ud = torch.from_numpy(u).cuda()
    fe = m.external_force(s_dev)
    out = m.assemble(s_dev, ud, "f64", f_ext=fe, dirichlet=torch.from_numpy(d).cuda())
    torch.cuda.synchronize()
    perm = to_np(m.arrays()["perm"])
    e_f = rel_err(to_np(out["f_int"]), ref["f_int"])
    e_k = rel_err(to_np(out["K"]), ref["K"])
    e_s = rel_err(to_np(out["sigma"]), ref["sigma"][:, perm])
    e_fe = rel_err(to_np(fe), fe_ref)
    e_r = rel_err(to_np(out["r"]), r_ref)
    e_rn = abs(float(to_np(out["rnorm"])[0]) - rn_ref) / rn_ref
    log(f"[parity] {tag} f={e_f:.2e} K={e_k:.2e} sigma={e_s:.2e} fext={e_fe:.2e} r={e_r:.2e} rnorm={e_rn:.2e}")
    assert e_f <= TOL64 and e_k <= TOL64 and e_s <= TOL64 and e_fe <= TOL64 and e_r <= TOL64 and e_rn <= TOL64


@pytest.mark.parametrize("tag,kind,jit", CASES)
def test_assemble_fp32k_error_bounds(tag, kind, jit):
    w = _work(tag, kind)
    o, m, ps = build_pair(w, jitter=jit)
    st, u, s_dev, nodes = _inputs(w, o, ps, m, u_amp=2e-3)
    ref = o.assemble(st, u)
    fe_ref = o.external_force(dict(st, g=(0.0, 0.0, -9.81)))
    d = W.dirichlet_dofs(nodes)
    from oracle.oracle import residual
    r_ref, rn_ref = residual(ref["f_int"], fe_ref, d)
    fe = m.external_force(s_dev)
    out = m.assemble(s_dev, torch.from_numpy(u).cuda(), "f32k", f_ext=fe, dirichlet=torch.from_numpy(d).cuda())
    torch.cuda.synchronize()
    perm = to_np(m.arrays()["perm"])
    pl = ref["plastic"][perm]
    e_f = rel_err(to_np(out["f_int"]), ref["f_int"])
    e_k = rel_err(to_np(out["K"]), ref["K"])
    e_s = rel_err(to_np(out["sigma"]), ref["sigma"][:, perm])
    e_r = rel_err(to_np(out["r"]), r_ref)
    e_rn = abs(float(to_np(out["rnorm"])[0]) - rn_ref) / rn_ref
    log(f"[parity] {tag} fp32k f={e_f:.2e} K={e_k:.2e} sigma={e_s:.2e} r={e_r:.2e} rnorm={e_rn:.2e} "
        f"plastic={pl.mean():.2f}")
    assert out["K"].dtype == torch.float32 and out["f_int"].dtype == torch.float64
    assert e_f <= TOL32_F and e_k <= TOL32_K and e_s <= TOL32_SIG and e_r <= TOL32_F and e_rn <= TOL32_F


@pytest.mark.parametrize("tag,kind,jit", [("c0", None, None), ("tiny_sphere_jit", "sphere", 0),
                                          ("tiny_cone_vm_jit", "cone", 1)])
def test_adjoint_matches_oracle(tag, kind, jit):
    w = _work(tag, kind)
    o, m, ps = build_pair(w, jitter=jit)
    st, u, s_dev, nodes = _inputs(w, o, ps, m, u_amp=2e-3)
    lam = W.make_lambda(w, nodes)
    ref = o.adjoint(st, u, lam)
    perm = to_np(m.arrays()["perm"])
    ud, ld = torch.from_numpy(u).cuda(), torch.from_numpy(lam).cuda()
    for prec, tol in (("f64", TOL64), ("f32k", 2e-4)):
        g = m.adjoint(s_dev, ud, ld, prec)
        torch.cuda.synchronize()
        errs = {k: rel_err(to_np(g[k]), ref[k][perm]) for k in ("dE", "dnu", "dsy", "dV")}
        log(f"[parity] {tag} adjoint {prec} " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
        assert all(v <= tol for v in errs.values()), errs


def test_autograd_function_matches_adjoint():
    from paper_2606_09275_amd.autograd import MPMForce
    w = tiny_workload("sphere", E=1e4, nu=0.3, sy=40.0, Fn_std=0.03)
    o, m, ps = build_pair(w, jitter=0)
    st, u, s_dev, nodes = _inputs(w, o, ps, m, u_amp=2e-3)
    lam = torch.from_numpy(W.make_lambda(w, nodes)).cuda()
    params = {k: s_dev[k].reshape(-1).clone().requires_grad_(True) for k in ("E", "nu", "sy", "vol")}
    rest = {k: v for k, v in s_dev.items() if k not in params}
    f = MPMForce.apply(m, rest, torch.from_numpy(u).cuda(), params["E"], params["nu"], params["sy"], params["vol"])
    L = (f * lam).sum()
    L.backward()
    ref = o.adjoint(st, u, to_np(lam))
    perm = to_np(m.arrays()["perm"])
    for k, key in (("E", "dE"), ("nu", "dnu"), ("sy", "dsy"), ("vol", "dV")):
        assert rel_err(to_np(params[k].grad), ref[key][perm]) <= TOL64


def test_c1_full_size_parity():
    """C1 at full size: mesh/order/CSR bit-exact and every output against the oracle."""
    w = W.get("c1")
    o, m, ps = build_pair(w)
    _mesh_checks(o, m, ps)
    st, u, s_dev, nodes = _inputs(w, o, ps, m)
    ref = o.assemble(st, u)
    perm = to_np(m.arrays()["perm"])
    out = m.assemble(s_dev, torch.from_numpy(u).cuda(), "f64", commit=True)
    torch.cuda.synchronize()
    e = (rel_err(to_np(out["f_int"]), ref["f_int"]), rel_err(to_np(out["K"]), ref["K"]),
         rel_err(to_np(out["sigma"]), ref["sigma"][:, perm]), rel_err(to_np(out["F_new"]), ref["Fnew"][:, perm]),
         rel_err(to_np(out["be_new"]), ref["be"][:, perm]))
    log(f"[parity] c1 full fp64 f={e[0]:.2e} K={e[1]:.2e} sigma={e[2]:.2e} F_new={e[3]:.2e} b_e={e[4]:.2e} "
        f"plastic={ref['plastic'].mean():.3f}")
    assert max(e) <= TOL64
    out32 = m.assemble(s_dev, torch.from_numpy(u).cuda(), "f32k")
    torch.cuda.synchronize()
    e32 = (rel_err(to_np(out32["f_int"]), ref["f_int"]), rel_err(to_np(out32["K"]), ref["K"]))
    log(f"[parity] c1 full fp32k f={e32[0]:.2e} K={e32[1]:.2e}")
    assert e32[0] <= TOL32_F and e32[1] <= TOL32_K
