"""GPU parity of the Newton-step solve through the C ABI: y = K x against a CPU sparse product
of the same values (FP64 and FP32 tangents), and the Jacobi-preconditioned CG solution against
the CPU direct solve of the reduced system (and the CPU iteration's count), on tangents the
library assembled; zero right-hand side; the full-size cone-penetration tangent."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle.solve import jacobi_pcg, reduced_solve, csr
from tests.gpu_common import build_pair, log, rel_err, to_np
from tests.helpers import tiny_workload

pytestmark = pytest.mark.gpu


def _assembled(kind, jit, sy, prec):
    w = tiny_workload(kind, E=1e4, nu=0.3, sy=sy, Fn_std=0.02)
    o, m, ps = build_pair(w, jitter=jit, oracle_points=False)
    st = W.make_state(w, ps)
    nodes = to_np(m.arrays()["node_ijk"])
    u = torch.from_numpy(W.make_u(w, nodes, amp=1e-4)).cuda()
    d = torch.from_numpy(W.dirichlet_dofs(nodes)).cuda()
    out = m.assemble(m.sorted_state(st), u, prec)
    torch.cuda.synchronize()
    a = m.arrays()
    A = csr(to_np(a["row_ptr"]), to_np(a["col"]), to_np(out["K"]).astype(np.float64), m.info["n_dof"])
    return m, out, d, A


@pytest.mark.parametrize("prec", ["f64", "f32k"])
@pytest.mark.parametrize("kind,jit,sy", [("sphere", None, math.inf), ("cone", 1, 5.0)])
def test_spmv_matches_cpu_product(kind, jit, sy, prec):
    m, out, d, A = _assembled(kind, jit, sy, prec)
    rng = np.random.default_rng(7)
    x = rng.normal(size=m.info["n_dof"])
    y = to_np(m.spmv(out["K"], torch.from_numpy(x).cuda()))
    ref = A @ x
    e = rel_err(y, ref)
    log(f"[parity] spmv {kind} {prec}: {e:.2e}")
    assert e <= 1e-14


@pytest.mark.parametrize("prec,tol", [("f64", 1e-7), ("f32k", 1e-6)])
def test_cg_matches_direct_solve(prec, tol):
    m, out, d, A = _assembled("sphere", None, math.inf, prec)
    b = -to_np(out["f_int"])
    dn = to_np(d)
    x, it, rel = m.solve_cg(out["K"], torch.from_numpy(b).cuda(), d, rtol=1e-12, max_iter=20000)
    torch.cuda.synchronize()
    xd = reduced_solve(A, b, dn)
    xc, itc, relc = jacobi_pcg(A, b, dn, rtol=1e-12, max_iter=20000)
    e = rel_err(to_np(x), xd)
    log(f"[parity] cg {prec}: iterations {it} (cpu {itc}), relres {rel:.2e}, x vs direct {e:.2e}")
    assert rel <= 1e-12 and e <= tol
    assert abs(it - itc) <= max(3, itc // 50)
    assert np.all(to_np(x)[dn.astype(bool)] == 0.0)


def test_cg_zero_rhs_and_iteration_cap():
    m, out, d, A = _assembled("box", 2, 5.0, "f64")
    zero = torch.zeros(m.info["n_dof"], dtype=torch.float64, device="cuda")
    x, it, rel = m.solve_cg(out["K"], zero, d)
    assert it == 0 and float(x.abs().max()) == 0.0
    b = torch.from_numpy(-to_np(out["f_int"])).cuda()
    x, it, rel = m.solve_cg(out["K"], b, d, rtol=1e-30, max_iter=5)
    assert it == 5 and rel > 0.0


def test_spmv_full_size_cone_tangent():
    """SpMV on the 54.4M-entry tangent of the cone-penetration workload against the CPU
    product of the same values."""
    from paper_2606_09275_amd.mesh import Mesh
    w = W.get("c2")
    m0 = Mesh(w.crit())
    lv = to_np(m0.arrays()["leaf"])
    del m0
    ps = W.make_points(w, lv[:, :3], lv[:, 3])
    m = Mesh(w.crit(), torch.from_numpy(ps.x).cuda(), torch.from_numpy(ps.l).cuda())
    st = W.make_state(w, ps)
    nodes = to_np(m.arrays()["node_ijk"])
    u = torch.from_numpy(W.make_u(w, nodes)).cuda()
    out = m.assemble(m.sorted_state(st), u, "f64", want_sigma=False)
    a = m.arrays()
    A = csr(to_np(a["row_ptr"]), to_np(a["col"]), to_np(out["K"]), m.info["n_dof"])
    x = np.random.default_rng(8).normal(size=m.info["n_dof"])
    y = to_np(m.spmv(out["K"], torch.from_numpy(x).cuda()))
    e = rel_err(y, A @ x)
    log(f"[parity] spmv c2 full: {e:.2e}")
    assert e <= 1e-14
