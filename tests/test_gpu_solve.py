"""GPU parity of the Newton-step solves through the C ABI. The solver inputs are the oracle's:
its assembled tangent, or seeded normal values on its CSR pattern (which the library's mesh
reproduces bit-exactly), uploaded in the precision under test. y = K x against the CPU sparse
product; Jacobi-preconditioned CG and restarted GMRES against the CPU direct solve of the
reduced system and against the oracle iterations (iteration counts; GMRES iterates step by
step); a non-symmetric (row-scaled) and an indefinite (shifted) tangent for GMRES; zero
right-hand side, zero budget and argument limits; the full-size cone-penetration tangent."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle.solve import csr, free_dofs, jacobi_gmres, jacobi_pcg, reduced_solve
from paper_2606_09275_amd._lib import MPMError
from tests.gpu_common import build_pair, log, rel_err, to_np
from tests.helpers import tiny_workload

pytestmark = pytest.mark.gpu


def _system(kind, jit, sy, prec, values="oracle"):
    """Library mesh on the oracle's points, K values on the oracle's CSR pattern (its elastic
    tangent and -f_int, or seeded normal values), the CPU matrix of the same values and the
    Dirichlet mask of the fixed base."""
    w = tiny_workload(kind, E=1e4, nu=0.3, sy=sy, Fn_std=0.02)
    o, m, ps = build_pair(w, jitter=jit)
    rp, col = o.csr()
    a = m.arrays()
    assert np.array_equal(to_np(a["row_ptr"]), rp) and np.array_equal(to_np(a["col"]), col)
    nodes = o.nodes()
    ndof = 3 * nodes.shape[0]
    if values == "oracle":
        ref = o.assemble(W.make_state(w, ps), W.make_u(w, nodes, amp=1e-4))
        kv, b = ref["K"], -ref["f_int"]
    else:
        rng = np.random.default_rng(5)
        kv, b = rng.normal(size=col.size), rng.normal(size=ndof)
    K = torch.from_numpy(np.ascontiguousarray(kv)).to(torch.float64 if prec == "f64" else torch.float32).cuda()
    A = csr(rp, col, to_np(K).astype(np.float64), ndof)
    return m, K, A, b, W.dirichlet_dofs(nodes)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("prec", ["f64", "f32k"])
@pytest.mark.parametrize("kind,jit,sy", [("sphere", None, math.inf), ("cone", 1, 5.0)])
def test_spmv_matches_cpu_product(kind, jit, sy, prec):
    m, K, A, _, _ = _system(kind, jit, sy, prec, values="random")
    x = np.random.default_rng(7).normal(size=A.shape[0])
    y = to_np(m.spmv(K, _cuda(x)))
    e = rel_err(y, A @ x)
    log(f"[parity] spmv {kind} {prec}: {e:.2e}")
    assert e <= 1e-14


@pytest.mark.parametrize("prec,tol", [("f64", 1e-7), ("f32k", 1e-6)])
def test_cg_matches_direct_solve(prec, tol):
    m, K, A, b, dn = _system("sphere", None, math.inf, prec)
    x, it, rel = m.solve_cg(K, _cuda(b), _cuda(dn), rtol=1e-12, max_iter=20000)
    torch.cuda.synchronize()
    xd = reduced_solve(A, b, dn)
    xc, itc, relc = jacobi_pcg(A, b, dn, rtol=1e-12, max_iter=20000)
    e = rel_err(to_np(x), xd)
    log(f"[parity] cg {prec}: iterations {it} (cpu {itc}), relres {rel:.2e}, x vs direct {e:.2e}")
    assert rel <= 1e-12 and e <= tol
    assert abs(it - itc) <= max(3, itc // 50)
    assert np.all(to_np(x)[dn.astype(bool)] == 0.0)


def test_cg_zero_rhs_and_iteration_cap():
    m, K, A, b, dn = _system("box", 2, 5.0, "f64")
    d = _cuda(dn)
    zero = torch.zeros(A.shape[0], dtype=torch.float64, device="cuda")
    x, it, rel = m.solve_cg(K, zero, d)
    assert it == 0 and float(x.abs().max()) == 0.0
    x, it, rel = m.solve_cg(K, _cuda(b), d, rtol=1e-30, max_iter=5)
    assert it == 5 and rel > 0.0


def _fixed_zero(x, dn):
    return bool(np.all(to_np(x)[dn.astype(bool)] == 0.0))


@pytest.mark.parametrize("prec,tol", [("f64", 1e-7), ("f32k", 1e-6)])
def test_gmres_matches_direct_solve(prec, tol):
    m, K, A, b, dn = _system("sphere", None, math.inf, prec)
    x, it, rel = m.solve_gmres(K, _cuda(b), _cuda(dn), rtol=1e-12, restart=30, max_iter=20000)
    torch.cuda.synchronize()
    xd = reduced_solve(A, b, dn)
    xc, itc, relc = jacobi_gmres(A, b, dn, rtol=1e-12, restart=30, max_iter=20000)
    e = rel_err(to_np(x), xd)
    log(f"[parity] gmres {prec}: steps {it} (cpu {itc}), relres {rel:.2e} (cpu {relc:.2e}), x vs direct {e:.2e}")
    assert rel <= 1e-12 and e <= tol
    assert abs(it - itc) <= max(3, itc // 50)
    assert _fixed_zero(x, dn)


@pytest.mark.parametrize("restart,steps", [(1, 7), (5, 12), (30, 40), (64, 70)])
def test_gmres_iterates_match_oracle(restart, steps):
    """A fixed number of Arnoldi steps (no convergence test): the iterate after those steps and
    its true residual against the oracle's, through restarts and a partial last cycle."""
    m, K, A, b, dn = _system("sphere", None, math.inf, "f64")
    x, it, rel = m.solve_gmres(K, _cuda(b), _cuda(dn), rtol=0.0, restart=restart, max_iter=steps)
    torch.cuda.synchronize()
    xc, itc, relc = jacobi_gmres(A, b, dn, rtol=0.0, restart=restart, max_iter=steps)
    e = rel_err(to_np(x), xc)
    log(f"[parity] gmres({restart}) after {steps} steps: x vs oracle {e:.2e}, relres {rel:.6e} / {relc:.6e}")
    assert it == itc == steps
    assert e <= 1e-9 and abs(rel - relc) <= 1e-9 * relc
    assert _fixed_zero(x, dn)


def test_gmres_nonsymmetric_row_scaled():
    """D K x = D b with a seeded positive row scaling D: a non-symmetric system with the
    solution of K x = b."""
    m, K, A, b, dn = _system("sphere", None, math.inf, "f64")
    n = A.shape[0]
    D = np.random.default_rng(9).uniform(0.5, 2.0, size=n)
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    Ks = to_np(K) * D[rows]
    As = csr(A.indptr, A.indices, Ks, n)
    assert abs(As - As.T).max() > 0.05 * abs(As).max()
    x, it, rel = m.solve_gmres(_cuda(Ks), _cuda(D * b), _cuda(dn), rtol=1e-11, restart=30, max_iter=20000)
    torch.cuda.synchronize()
    xd = reduced_solve(A, b, dn)
    xc, itc, relc = jacobi_gmres(As, D * b, dn, rtol=1e-11, restart=30, max_iter=20000)
    e = rel_err(to_np(x), xd)
    log(f"[parity] gmres row-scaled: steps {it} (cpu {itc}), relres {rel:.2e}, x vs direct {e:.2e}")
    assert rel <= 1e-11 and e <= 1e-6
    assert abs(it - itc) <= max(3, itc // 50)


def test_gmres_indefinite_where_cg_stops():
    """The tangent minus 2 % of its diagonal is indefinite on the free DOFs: CG ends without
    converging, GMRES reaches the direct solution."""
    m, K, A, b, dn = _system("sphere", None, math.inf, "f64")
    n = A.shape[0]
    kv = to_np(K).copy()
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    kv[A.indices == rows] *= 0.98
    Ai = csr(A.indptr, A.indices, kv, n)
    Ki, bd, d = _cuda(kv), _cuda(b), _cuda(dn)
    _, it_cg, rel_cg = m.solve_cg(Ki, bd, d, rtol=1e-10, max_iter=20000)
    x, it, rel = m.solve_gmres(Ki, bd, d, rtol=1e-10, restart=30, max_iter=20000)
    torch.cuda.synchronize()
    xd = reduced_solve(Ai, b, dn)
    xc, itc, relc = jacobi_gmres(Ai, b, dn, rtol=1e-10, restart=30, max_iter=20000)
    e = rel_err(to_np(x), xd)
    log(f"[parity] indefinite: cg {it_cg} steps relres {rel_cg:.2e}; gmres {it} (cpu {itc}) relres {rel:.2e}, "
        f"x vs direct {e:.2e}")
    assert rel_cg > 1e-6
    assert rel <= 1e-10 and e <= 1e-6
    assert abs(it - itc) <= max(3, itc // 50)


def test_gmres_edges():
    m, K, A, b, dn = _system("box", 2, 5.0, "f64")
    d = _cuda(dn)
    zero = torch.zeros(A.shape[0], dtype=torch.float64, device="cuda")
    x, it, rel = m.solve_gmres(K, zero, d)
    assert it == 0 and rel == 0.0 and float(x.abs().max()) == 0.0
    x, it, rel = m.solve_gmres(K, _cuda(b), d, max_iter=0)
    assert it == 0 and rel == 1.0 and float(x.abs().max()) == 0.0
    for bad in (0, 65):
        with pytest.raises(MPMError):
            m.solve_gmres(K, _cuda(b), d, restart=bad)


def test_gmres_invariant_space_one_step():
    """Only the diagonal entries of the pattern set (seeded positive values): K M^-1 = I on the
    free DOFs, the first Arnoldi vector spans an invariant space (the new column vanishes up to
    rounding) and GMRES ends after one step with x = b / diag, as the oracle does."""
    m, K, A, b, dn = _system("sphere", None, math.inf, "f64", values="random")
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    kv = np.zeros(A.indices.size)
    diag = A.indices == rows
    kv[diag] = np.random.default_rng(21).uniform(1.0, 3.0, size=int(diag.sum()))
    Ad = csr(A.indptr, A.indices, kv, n)
    x, it, rel = m.solve_gmres(_cuda(kv), _cuda(b), _cuda(dn), rtol=1e-14, restart=30, max_iter=100)
    torch.cuda.synchronize()
    xc, itc, relc = jacobi_gmres(Ad, b, dn, rtol=1e-14, restart=30, max_iter=100)
    f = free_dofs(Ad, dn)
    xd = np.where(f, b / np.where(f, Ad.diagonal(), 1.0), 0.0)
    e = rel_err(to_np(x), xd)
    log(f"[parity] gmres diagonal: steps {it} (cpu {itc}), relres {rel:.2e}, x vs b/diag {e:.2e}")
    assert it == itc == 1 and rel <= 1e-15 and e <= 1e-15


def test_spmv_full_size_cone_tangent():
    """SpMV at the full size of the cone-penetration workload (54.4M values): seeded normal
    values on the oracle's CSR pattern of that mesh and its points, against the CPU product."""
    from oracle.oracle import OracleMesh
    from paper_2606_09275_amd.mesh import Mesh
    w = W.get("c2")
    o = OracleMesh(w.crit())
    lv = o.leaves()
    ps = W.make_points(w, lv[:, :3], lv[:, 3])
    o.set_points(ps.x, ps.l)
    rp, col = o.csr()
    m = Mesh(w.crit(), torch.from_numpy(ps.x).cuda(), torch.from_numpy(ps.l).cuda())
    a = m.arrays()
    assert np.array_equal(to_np(a["row_ptr"]), rp) and np.array_equal(to_np(a["col"]), col)
    ndof = m.info["n_dof"]
    rng = np.random.default_rng(8)
    kv = rng.normal(size=col.size)
    x = rng.normal(size=ndof)
    A = csr(rp, col, kv, ndof)
    y = to_np(m.spmv(_cuda(kv), _cuda(x)))
    e = rel_err(y, A @ x)
    log(f"[parity] spmv c2 full ({col.size} values): {e:.2e}")
    assert e <= 1e-14
