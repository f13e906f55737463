"""Pins of the CPU reference for the Newton-step solve: the free-DOF reduction (Dirichlet and
empty rows constrained out), closed forms on diagonal systems, the finite termination of
conjugate gradients (at most as many iterations as distinct eigenvalues), agreement of the
preconditioned iteration with the direct solve, and the assembled tangent of an elastic
problem (positive definite once the base is fixed)."""
import math

import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle.solve import free_dofs, jacobi_pcg, reduced_solve
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
