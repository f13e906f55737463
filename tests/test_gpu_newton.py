"""A whole Newton-Raphson load step (Section 2.4: residual, consistent tangent, linear solve,
update) run through the C ABI: body force f_ext, the base of the mesh fixed (Dirichlet), from
u = 0 each iteration assembles f_int and K on the GPU, solves K_ff du_f = -r_f by the
Jacobi-preconditioned CG and updates u. The same loop on the CPU takes the oracle's assembly
and a direct sparse solve of the reduced system. Both must converge (the tangent is the exact
Jacobian, so the residual falls quadratically) to the same displacement."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle.oracle import residual
from oracle.solve import csr, reduced_solve
from tests.gpu_common import build_pair, log, rel_err, to_np
from tests.helpers import tiny_workload

pytestmark = pytest.mark.gpu

MAX_IT = 10
RTOL = 1e-10


def _cpu_newton(o, st, g, d, nd):
    u = np.zeros(3 * nd)
    fe = o.external_force(dict(st, g=g))
    hist = []
    for _ in range(MAX_IT):
        ref = o.assemble(st, u)
        r, rn = residual(ref["f_int"], fe, d)
        hist.append(rn)
        if rn <= RTOL * hist[0]:
            break
        rp, col = o.csr()
        A = csr(rp, col, ref["K"], 3 * nd)
        u = u + reduced_solve(A, -r, d)
    return u, hist


# elastic: a body force 20 g (strains near 1e-2, geometric nonlinearity); von Mises: committed
# deformation gradients I + N(0, 0.02^2) and sigma_y = 15, so that nearly every point returns
# to the yield surface (the plastic branch of the tangent)
@pytest.mark.parametrize("tag,E,sy,gscale,fn_std", [("elastic", 1e3, math.inf, 20.0, 0.0),
                                                    ("vm", 1e3, 15.0, 1.0, 0.02)])
def test_newton_load_step_matches_cpu(tag, E, sy, gscale, fn_std):
    w = tiny_workload("sphere", E=E, nu=0.3, sy=sy, Fn_std=fn_std)
    o, m, ps = build_pair(w)
    st = W.make_state(w, ps)
    g = (0.0, 0.0, -9.81 * gscale)
    nodes = o.nodes()
    nd = nodes.shape[0]
    d = W.dirichlet_dofs(nodes)
    u_cpu, h_cpu = _cpu_newton(o, st, g, d, nd)

    s_dev = m.sorted_state(dict(st, g=g))
    fe = m.external_force(s_dev)
    dd = torch.from_numpy(d).cuda()
    u = torch.zeros(3 * nd, dtype=torch.float64, device="cuda")
    hist, cg_its = [], []
    out = {}
    for _ in range(MAX_IT):
        m.assemble(s_dev, u, "f64", f_ext=fe, dirichlet=dd, out=out)
        rn = float(to_np(out["rnorm"])[0])
        hist.append(rn)
        if rn <= RTOL * hist[0]:
            break
        du, it, rel = m.solve_cg(out["K"], -out["r"], dd, rtol=1e-13, max_iter=50000)
        assert rel <= 1e-13, (it, rel)
        cg_its.append(it)
        u += du
    torch.cuda.synchronize()
    plastic = float(o.assemble(st, u_cpu)["plastic"].mean())
    log(f"[newton] {tag}: gpu residuals {' '.join(f'{v:.1e}' for v in hist)} (cg {cg_its}); "
        f"cpu {' '.join(f'{v:.1e}' for v in h_cpu)}; plastic fraction {plastic:.2f}")
    assert hist[-1] <= RTOL * hist[0] and h_cpu[-1] <= RTOL * h_cpu[0]
    assert len(hist) == len(h_cpu)
    # the iterations of the two loops agree while the residual is far above the solve accuracy
    for a, b in zip(hist[:3], h_cpu[:3]):
        assert abs(a - b) <= 1e-6 * h_cpu[0] + 1e-3 * b
    e_u = rel_err(to_np(u), u_cpu)
    log(f"[parity] newton {tag}: u vs cpu {e_u:.2e}, max |u| {np.abs(u_cpu).max():.3e}")
    assert e_u <= 1e-8
    if tag == "vm":
        assert plastic > 0.0
