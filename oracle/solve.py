"""CPU reference for the linear solve of a Newton step (test infrastructure only).

Only tests and the benchmark may import this module; the library never does.

The Newton step solves K du = -r with the Dirichlet DOFs constrained out of the system
(Section 2.4, strong treatment): over the free DOFs f (not Dirichlet, row not empty,
positive diagonal) K_ff x_f = b_f, x = 0 elsewhere.

* reduced_solve: that definition, with a sparse direct solve (scipy's LU) as the step;
* jacobi_pcg: textbook preconditioned conjugate gradients with M = diag(K_ff), the same
  stopping rule as the GPU solver (||r|| <= rtol ||b_f||), in plain numpy.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def csr(row_ptr, col, vals, ndof):
    return sp.csr_matrix((np.asarray(vals, dtype=np.float64), np.asarray(col), np.asarray(row_ptr)),
                         shape=(ndof, ndof))


def free_dofs(A: sp.csr_matrix, dirichlet=None) -> np.ndarray:
    """Free DOFs: not Dirichlet, non-empty row, positive diagonal."""
    nonempty = np.diff(A.indptr) > 0
    diag = A.diagonal()
    f = nonempty & (diag > 0)
    if dirichlet is not None:
        f &= ~np.asarray(dirichlet, dtype=bool)
    return f


def reduced_solve(A: sp.csr_matrix, b: np.ndarray, dirichlet=None) -> np.ndarray:
    f = free_dofs(A, dirichlet)
    idx = np.nonzero(f)[0]
    x = np.zeros(A.shape[0])
    if idx.size:
        Aff = A[idx][:, idx].tocsc()
        x[idx] = spla.spsolve(Aff, np.asarray(b, dtype=np.float64)[idx])
    return x


def jacobi_pcg(A: sp.csr_matrix, b: np.ndarray, dirichlet=None, rtol=1e-8, max_iter=1000):
    """Returns (x, iterations, ||r|| / ||b_f||)."""
    f = free_dofs(A, dirichlet)
    idx = np.nonzero(f)[0]
    Aff = A[idx][:, idx]
    bf = np.asarray(b, dtype=np.float64)[idx]
    dinv = 1.0 / Aff.diagonal()
    x = np.zeros_like(bf)
    r = bf.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    bb = bf @ bf
    it = 0
    if bb > 0:
        while it < max_iter:
            q = Aff @ p
            pq = p @ q
            if not pq > 0:
                break
            alpha = rz / pq
            x += alpha * p
            r -= alpha * q
            z = dinv * r
            rz_new = r @ z
            it += 1
            if not (r @ r > rtol * rtol * bb) or not rz_new > 0:
                break
            p = z + (rz_new / rz) * p
            rz = rz_new
    out = np.zeros(A.shape[0])
    out[idx] = x
    rel = float(np.sqrt((r @ r) / bb)) if bb > 0 else 0.0
    return out, it, rel
