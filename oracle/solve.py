"""CPU reference for the linear solve of a Newton step (test infrastructure only).

Only tests and the benchmark may import this module; the library never does.

The Newton step solves K du = -r with the Dirichlet DOFs constrained out of the system
(Section 2.4, strong treatment): over the free DOFs f (not Dirichlet, row not empty,
positive diagonal) K_ff x_f = b_f, x = 0 elsewhere.

* reduced_solve: that definition, with a sparse direct solve (scipy's LU) as the step;
* jacobi_pcg: textbook preconditioned conjugate gradients with M = diag(K_ff), the same
  stopping rule as the GPU solver (||r|| <= rtol ||b_f||), in plain numpy;
* jacobi_gmres: restarted GMRES (the Krylov solver the paper names for its possibly
  non-symmetric systems, Sections 1 and 6, with the diagonal Jacobi preconditioner it proposes
  there), preconditioned on the right, so that the minimised quantity is the true residual
  ||b_f - K_ff x_f||. Written from the published algorithm of Saad and Schultz (1986): the
  Arnoldi process with modified Gram-Schmidt, the Hessenberg least-squares problem reduced by
  Givens rotations as the columns arrive, the correction x += M^-1 V_k y at the end of a cycle,
  and the true residual recomputed at each restart.
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


def jacobi_gmres(A: sp.csr_matrix, b: np.ndarray, dirichlet=None, rtol=1e-8, restart=30, max_iter=1000,
                 history=False):
    """Returns (x, iterations, ||b_f - K_ff x_f|| / ||b_f||) and, with history=True, also the
    list of residual norms that the rotations give after each Arnoldi step. A cycle ends after
    `restart` steps, when the rotated residual falls to rtol ||b_f||, at max_iter steps in
    all, or when the Krylov space becomes invariant (new column of norm zero); the solve stops
    when the recomputed residual meets the tolerance or the step budget is spent."""
    f = free_dofs(A, dirichlet)
    idx = np.nonzero(f)[0]
    Aff = A[idx][:, idx]
    bf = np.asarray(b, dtype=np.float64)[idx]
    dinv = 1.0 / Aff.diagonal()
    m = int(restart)
    x = np.zeros_like(bf)
    bnorm = float(np.linalg.norm(bf))
    hist = []
    it = 0
    r = bf.copy()
    beta = bnorm
    while beta > rtol * bnorm and it < max_iter:
        V = np.zeros((m + 1, bf.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = Aff @ (dinv * V[j])
            for i in range(j + 1):  # modified Gram-Schmidt against the basis so far
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            hn = float(np.linalg.norm(w))
            H[j + 1, j] = hn
            for i in range(j):  # earlier rotations, in order, on the new column
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            d = float(np.hypot(H[j, j], H[j + 1, j]))
            cs[j], sn[j] = H[j, j] / d, H[j + 1, j] / d
            H[j, j], H[j + 1, j] = d, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            hist.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= rtol * bnorm or it >= max_iter or hn == 0.0:
                break
            V[j + 1] = w / hn
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):  # back substitution in the triangular H[:k, :k]
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + dinv * (V[:k].T @ y)
        r = bf - Aff @ x
        beta = float(np.linalg.norm(r))
    out = np.zeros(A.shape[0])
    out[idx] = x
    rel = beta / bnorm if bnorm > 0 else 0.0
    return (out, it, rel, hist) if history else (out, it, rel)
