"""Pins of the CPU reference for the Newton-step solve: the free-DOF reduction (Dirichlet and
empty rows constrained out), closed forms on diagonal systems, the finite termination of
conjugate gradients (at most as many iterations as distinct eigenvalues), agreement of the
preconditioned iteration with the direct solve, and the assembled tangent of an elastic
problem (positive definite once the base is fixed). GMRES: finite termination on a dense
non-symmetric system, the minimal-residual property (each step's rotated residual equals the
least-squares minimum over the Krylov space, computed from an explicit Krylov basis), restarts
with Dirichlet DOFs on a non-symmetric sparse system, and an indefinite tangent on which
conjugate gradients break down."""
import math

import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle.solve import free_dofs, jacobi_gmres, jacobi_pcg, reduced_solve
from tests.helpers import setup, tiny_workload


def test_diagonal_system_closed_form():
    d = np.array([2.0, 0.0, 5.0, 4.0, 1.0])
    A = sp.csr_matrix(np.diag(d))
    b = np.array([1.0, 7.0, -3.0, 8.0, 2.0])
    dirichlet = np.array([0, 0, 0, 1, 0], dtype=np.uint8)
    f = free_dofs(A, dirichlet)
    assert f.tolist() == [True, False, True, False, True]
    x = reduced_solve(A, b, dirichlet)
    assert np.allclose(x, [0.5, 0.0, -0.6, 0.0, 2.0], rtol=0, atol=1e-15)
    xc, it, rel = jacobi_pcg(A, b, dirichlet, rtol=1e-14)
    assert it == 1 and np.allclose(xc, x, rtol=0, atol=1e-15) and rel < 1e-14


def test_cg_terminates_in_distinct_eigenvalue_count():
    """A = B (x) I_10 + 0.1 I_3 (x) J_10 (J all ones) has a constant diagonal, so the Jacobi
    preconditioner is a multiple of the identity, and commuting terms give exactly four
    distinct eigenvalues ({3, 1.5} + {0, 1}): conjugate gradients end in four iterations."""
    B = np.array([[2.0, 0.5, 0.5], [0.5, 2.0, 0.5], [0.5, 0.5, 2.0]])
    A = np.kron(B, np.eye(10)) + 0.1 * np.kron(np.eye(3), np.ones((10, 10)))
    assert np.allclose(np.unique(np.round(np.linalg.eigvalsh(A), 10)), [1.5, 2.5, 3.0, 4.0])
    A = sp.csr_matrix(A)
    rng = np.random.default_rng(4)
    b = rng.normal(size=30)
    x, it, rel = jacobi_pcg(A, b, rtol=1e-12, max_iter=100)
    assert it == 4 and rel < 1e-12
    assert np.abs(x - reduced_solve(A, b)).max() < 1e-12 * np.abs(x).max()


def test_pcg_matches_direct_solve_on_elastic_tangent():
    w = tiny_workload("sphere", E=1e4, nu=0.3, sy=math.inf)
    m, ps = setup(w)
    s = W.make_state(w, ps)
    nodes = m.nodes()
    u = W.make_u(w, nodes, amp=1e-4)
    out = m.assemble(s, u)
    rp, col = m.csr()
    A = sp.csr_matrix((out["K"], col, rp), shape=(u.size, u.size))
    d = W.dirichlet_dofs(nodes)
    b = -out["f_int"]
    xd = reduced_solve(A, b, d)
    f = free_dofs(A, d)
    # the direct solution satisfies the reduced equations and vanishes on the fixed DOFs
    res = (A @ xd - b)[f]
    assert np.abs(res).max() < 1e-10 * np.abs(b[f]).max()
    assert np.all(xd[~f] == 0.0)
    xc, it, rel = jacobi_pcg(A, b, d, rtol=1e-12, max_iter=5000)
    assert rel < 1e-12 and 0 < it < 5000
    assert np.abs(xc - xd).max() < 1e-7 * np.abs(xd).max()
    # symmetric positive definite on the free DOFs
    Aff = A[np.nonzero(f)[0]][:, np.nonzero(f)[0]]
    assert abs(Aff - Aff.T).max() < 1e-10 * abs(Aff).max()
    assert sp.linalg.eigsh(Aff, k=1, which="SA", return_eigenvectors=False)[0] > 0


def test_gmres_finite_termination_dense_nonsymmetric():
    """Without restarts GMRES reaches the exact solution in at most n steps."""
    rng = np.random.default_rng(1)
    n = 10
    A = rng.normal(size=(n, n)) + 8.0 * np.eye(n)
    assert np.abs(A - A.T).max() > 1.0
    b = rng.normal(size=n)
    x, it, rel = jacobi_gmres(sp.csr_matrix(A), b, rtol=1e-14, restart=n, max_iter=n)
    xs = np.linalg.solve(A, b)
    assert it <= n and rel < 1e-13
    assert np.abs(x - xs).max() < 1e-12 * np.abs(xs).max()


def test_gmres_minimal_residual_property():
    """After k steps the iterate minimises ||b - A x|| over x in M^-1 K_k(A M^-1, b): the
    rotated residual of step k equals the least-squares minimum taken over an explicitly
    built (column-normalised) Krylov basis."""
    rng = np.random.default_rng(2)
    n = 40
    A = np.diag(rng.uniform(1.0, 4.0, size=n)) + 0.3 * rng.normal(size=(n, n))
    b = rng.normal(size=n)
    x, it, rel, hist = jacobi_gmres(sp.csr_matrix(A), b, rtol=1e-30, restart=n, max_iter=8, history=True)
    assert it == 8 and len(hist) == 8
    dinv = 1.0 / np.diag(A)
    B = A * dinv[None, :]  # A M^-1
    cols = [b / np.linalg.norm(b)]
    for k in range(1, 9):
        Kk = np.stack(cols, axis=1)
        y, *_ = np.linalg.lstsq(B @ Kk, b, rcond=None)
        best = np.linalg.norm(b - B @ Kk @ y)
        assert abs(hist[k - 1] - best) <= 1e-9 * np.linalg.norm(b), (k, hist[k - 1], best)
        v = B @ cols[-1]
        cols.append(v / np.linalg.norm(v))
    assert all(hist[k + 1] <= hist[k] * (1 + 1e-12) for k in range(7))
    # the returned iterate has the last step's residual
    assert abs(np.linalg.norm(b - A @ x) - hist[-1]) <= 1e-9 * np.linalg.norm(b)


def test_gmres_restarted_with_dirichlet_nonsymmetric():
    """Convection-diffusion stencil (-1 - c, 2, -1 + c): restarts every 4 steps, 5 fixed DOFs."""
    n, c = 60, 0.4
    A = sp.diags([np.full(n - 1, -1.0 - c), np.full(n, 2.0), np.full(n - 1, -1.0 + c)], [-1, 0, 1]).tocsr()
    rng = np.random.default_rng(3)
    b = rng.normal(size=n)
    d = np.zeros(n, dtype=np.uint8)
    d[[0, 7, 30, 31, 59]] = 1
    x, it, rel = jacobi_gmres(A, b, d, rtol=1e-11, restart=4, max_iter=5000)
    xd = reduced_solve(A, b, d)
    f = free_dofs(A, d)
    assert it > 4 and rel <= 1e-11
    assert np.linalg.norm((A @ x - b)[f]) <= 1e-11 * np.linalg.norm(b[f]) * (1 + 1e-6)
    assert np.all(x[~f] == 0.0)
    assert np.abs(x - xd).max() < 1e-8 * np.abs(xd).max()


def test_gmres_zero_rhs_and_zero_budget():
    A = sp.csr_matrix(np.diag([2.0, 3.0, 4.0]))
    x, it, rel = jacobi_gmres(A, np.zeros(3))
    assert it == 0 and rel == 0.0 and np.all(x == 0.0)
    x, it, rel = jacobi_gmres(A, np.ones(3), max_iter=0)
    assert it == 0 and rel == 1.0 and np.all(x == 0.0)
    # one step on a diagonal system with the Jacobi preconditioner is exact
    x, it, rel = jacobi_gmres(A, np.array([2.0, 6.0, -4.0]), rtol=1e-14)
    assert it == 1 and np.allclose(x, [1.0, 2.0, -1.0], rtol=0, atol=1e-15)


def test_gmres_indefinite_shifted_tangent():
    """The elastic tangent minus 2 % of its diagonal has negative eigenvalues on the free DOFs:
    conjugate gradients stop without converging, GMRES reaches the direct solution."""
    w = tiny_workload("sphere", E=1e4, nu=0.3, sy=math.inf)
    m, ps = setup(w)
    s = W.make_state(w, ps)
    nodes = m.nodes()
    u = W.make_u(w, nodes, amp=1e-4)
    out = m.assemble(s, u)
    rp, col = m.csr()
    A = sp.csr_matrix((out["K"], col, rp), shape=(u.size, u.size))
    A = sp.csr_matrix(A - 0.02 * sp.diags(A.diagonal()))
    d = W.dirichlet_dofs(nodes)
    b = -out["f_int"]
    f = np.nonzero(free_dofs(A, d))[0]
    assert sp.linalg.eigsh(A[f][:, f], k=1, which="SA", return_eigenvectors=False)[0] < 0
    xc, itc, relc = jacobi_pcg(A, b, d, rtol=1e-10, max_iter=20000)
    assert relc > 1e-6
    x, it, rel = jacobi_gmres(A, b, d, rtol=1e-10, restart=30, max_iter=20000)
    xd = reduced_solve(A, b, d)
    assert rel <= 1e-10 and np.abs(x - xd).max() < 1e-6 * np.abs(xd).max()
