"""Edge cases of the point count through the C ABI, against the oracle: a mesh with no points
(empty pattern, zero forces, empty outputs), a single point (one wavefront with one active
lane), and 65 points (a full wavefront and a second one holding one point). Mesh, point order
and CSR bit-exact; f_int, K, sigma and the adjoint within the FP64 parity tolerance (FP32K
within its bounds)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.oracle import OracleMesh
from tests.gpu_common import log, rel_err, to_np
from tests.helpers import tiny_workload

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 2e-5


@pytest.mark.parametrize("npts", [0, 1, 65])
def test_point_count_edges(npts):
    from paper_2606_09275_amd.mesh import Mesh
    w = tiny_workload("sphere", E=1e4, nu=0.3, sy=40.0, Fn_std=0.02)
    o = OracleMesh(w.crit())
    lv = o.leaves()
    full = W.make_points(w, lv[:, :3], lv[:, 3])
    # points from the middle of the generated set (several leaves, some with hanging nodes)
    s0 = full.n // 2
    ps = W.PointSet(x=np.ascontiguousarray(full.x[:, s0:s0 + npts]), l=np.ascontiguousarray(full.l[:, s0:s0 + npts]))
    o.set_points(ps.x, ps.l)
    log(f"[setup] {npts} points")
    m = Mesh(w.crit(), torch.from_numpy(ps.x).cuda(), torch.from_numpy(ps.l).cuda())
    a = m.arrays()
    rp, col = o.csr()
    assert m.info["n_point"] == npts and m.info["nnz"] == o.counts()["nnz"]
    assert np.array_equal(to_np(a["row_ptr"]), rp) and np.array_equal(to_np(a["col"]), col)
    perm_o, _, _ = o.perm()
    assert np.array_equal(to_np(a["perm"]), perm_o)

    st = W.make_state(w, ps)
    nodes = o.nodes()
    u = W.make_u(w, nodes, amp=2e-3)
    lam = W.make_lambda(w, nodes)
    ref = o.assemble(st, u)
    aref = o.adjoint(st, u, lam)
    s_dev = m.sorted_state(dict(st, g=(0.0, 0.0, -9.81)))
    ud, ld = torch.from_numpy(u).cuda(), torch.from_numpy(lam).cuda()
    perm = to_np(a["perm"])
    for prec, tol in (("f64", TOL64), ("f32k", TOL32)):
        out = m.assemble(s_dev, ud, prec)
        g = m.adjoint(s_dev, ud, ld, prec)
        torch.cuda.synchronize()
        errs = {
            "f": rel_err(to_np(out["f_int"]), ref["f_int"]),
            "K": rel_err(to_np(out["K"]), ref["K"]),
            "sigma": rel_err(to_np(out["sigma"]), ref["sigma"][:, perm]),
        }
        if prec == "f64":
            for k in ("dE", "dnu", "dsy", "dV"):
                errs[k] = rel_err(to_np(g[k]), aref[k][perm])
        log(f"[parity] {npts} points {prec}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
        assert all(v <= tol for v in errs.values()), errs
        if npts == 0:
            assert float(out["f_int"].abs().max()) == 0.0 and out["K"].numel() == 0
            assert out["sigma"].shape[1] == 0 and g["dE"].numel() == 0
