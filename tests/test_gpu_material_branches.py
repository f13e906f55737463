"""GPU parity of the material update on states that select its special branches: principal
logarithmic strains beyond the range of the small-argument series (the library then calls
log1p), exactly repeated eigenvalues (no rotation, theta at equal arguments), and eigenvector
rotations whose off-diagonal is so small against the diagonal gap that th^2 overflows (the
rotation tangent then comes from t = 1 / (2 |th|)). The oracle is the FP64 reference of the
same point arithmetic; tolerances as in the other FP64 parity tests."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_common import build_pair, log, rel_err, to_np
from tests.helpers import tiny_workload

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
SERIES_MAX = 1.0 / 16.0  # argument range of the series logarithm in the library


def _bn_eigs(bn):
    """eigenvalues of b_n - I per point, bn stored as (xx, yy, zz, xy, yz, xz)"""
    n = bn.shape[1]
    B = np.empty((n, 3, 3))
    B[:, 0, 0], B[:, 1, 1], B[:, 2, 2] = bn[0], bn[1], bn[2]
    B[:, 0, 1] = B[:, 1, 0] = bn[3]
    B[:, 1, 2] = B[:, 2, 1] = bn[4]
    B[:, 0, 2] = B[:, 2, 0] = bn[5]
    return np.linalg.eigvalsh(B - np.eye(3))


def _state(case, w, ps):
    st = W.make_state(w, ps)
    n = ps.n
    rng = np.random.default_rng(11)
    if case == "large_strain":
        pass  # F_n = I + N(0, 0.25^2): principal strains mostly beyond the series range
    elif case == "repeated":
        bn = np.zeros((6, n))
        bn[:3] = 1.0 + rng.choice([0.0, 2e-3], size=n)  # b_n = (1 + e) I: three equal eigenvalues
        st["bn"] = bn
        st["Jn"] = np.sqrt(bn[0] * bn[1] * bn[2])
    elif case == "tiny_offdiag":
        bn = np.zeros((6, n))
        bn[0], bn[1], bn[2] = 1.001, 1.002, 1.004
        # xy of normal size (the sweeps start), yz and xz tiny: after the (0,1) rotation the
        # (0,2) and (1,2) entries stay near 1e-220 against diagonal gaps near 1e-3
        bn[3] = rng.choice([-1.0, 1.0], size=n) * rng.uniform(1e-4, 5e-4, size=n)
        bn[4:] = rng.choice([-1.0, 1.0], size=(2, n)) * 10.0 ** rng.uniform(-250, -200, size=(2, n))
        st["bn"] = bn
        st["Jn"] = np.sqrt(bn[0] * bn[1] * bn[2])
    return st


CASES = [("large_strain", 0.25), ("repeated", 0.0), ("tiny_offdiag", 0.0)]


@pytest.mark.parametrize("case,fn_std", CASES)
def test_material_branches_match_oracle(case, fn_std):
    w = tiny_workload("sphere", E=1e4, nu=0.3, sy=40.0, Fn_std=fn_std)
    o, m, ps = build_pair(w)
    st = _state(case, w, ps)
    y = _bn_eigs(st["bn"])
    if case == "large_strain":
        frac = float((np.abs(y).max(axis=1) > SERIES_MAX).mean())
        log(f"[branch] {case}: points with a principal |b_n - I| beyond the series range: {frac:.2f}")
        assert frac > 0.5
    nodes = o.nodes()
    # displacements only where the state's own structure is not the point of the case
    u = W.make_u(w, nodes, amp=2e-3) if case == "large_strain" else np.zeros(3 * nodes.shape[0])
    lam = W.make_lambda(w, nodes)
    ref = o.assemble(st, u)
    aref = o.adjoint(st, u, lam)
    s_dev = m.sorted_state(dict(st, g=(0.0, 0.0, -9.81)))
    log(f"[run] {case} n={ps.n} plastic={ref['plastic'].mean():.2f}")
    ud, ld = torch.from_numpy(u).cuda(), torch.from_numpy(lam).cuda()
    out = m.assemble(s_dev, ud, "f64")
    g = m.adjoint(s_dev, ud, ld, "f64")
    torch.cuda.synchronize()
    perm = to_np(m.arrays()["perm"])
    errs = {
        "f": rel_err(to_np(out["f_int"]), ref["f_int"]),
        "K": rel_err(to_np(out["K"]), ref["K"]),
        "sigma": rel_err(to_np(out["sigma"]), ref["sigma"][:, perm]),
    }
    for k in ("dE", "dnu", "dsy", "dV"):
        errs[k] = rel_err(to_np(g[k]), aref[k][perm])
    log(f"[parity] {case} " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert all(v <= TOL64 for v in errs.values()), errs
