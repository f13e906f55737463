"""Pins of the oracle's assembly (weak form of Section 2.1): K against central differences
of f_int, balance of forces and moments, rigid-body invariances, symmetry, a patch test,
and the body-force term."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from tests.helpers import node_xyz, setup, tiny_workload


def _problem(kind, jit, sy, amp=2e-3, Fn_std=0.02):
    w = tiny_workload(kind, E=1e4, nu=0.3, sy=sy, Fn_std=Fn_std)
    m, ps = setup(w, jitter=jit)
    s = W.make_state(w, ps)
    u = W.make_u(w, m.nodes(), amp=amp)
    return w, m, ps, s, u


def _K(m, K):
    rp, col = m.csr()
    n = 3 * m.counts()["n_node"]
    return sp.csr_matrix((K, col, rp), shape=(n, n))


CASES = [("sphere", None, math.inf), ("sphere", 0, math.inf), ("cone", 1, 2.0), ("box", 2, 2.0), ("sphere", 3, 40.0)]


@pytest.mark.parametrize("kind,jit,sy", CASES)
def test_tangent_is_jacobian_of_internal_force(kind, jit, sy):
    w, m, ps, s, u = _problem(kind, jit, sy)
    out = m.assemble(s, u)
    if math.isfinite(sy) and sy < 10:
        assert out["plastic"].mean() > 0.9
    K = _K(m, out["K"])
    rng = np.random.default_rng(1)
    for _ in range(3):
        d = rng.normal(size=u.size)
        h = 1e-7
        fp = m.assemble(s, u + h * d, want_K=False)["f_int"]
        fm = m.assemble(s, u - h * d, want_K=False)["f_int"]
        fd = (fp - fm) / (2 * h)
        kd = K @ d
        assert np.abs(fd - kd).max() < 1e-6 * np.abs(kd).max()


@pytest.mark.parametrize("kind,jit,sy", CASES)
def test_balance_invariances_symmetry(kind, jit, sy):
    w, m, ps, s, u = _problem(kind, jit, sy)
    out = m.assemble(s, u)
    f = out["f_int"].reshape(-1, 3)
    K = _K(m, out["K"])
    scale = np.abs(f).max()
    assert np.abs(f.sum(axis=0)).max() < 1e-12 * np.abs(f).sum()           # sum of forces
    xc = node_xyz(w, m.nodes()) + u.reshape(-1, 3)
    mom = np.cross(xc, f).sum(axis=0)
    assert np.abs(mom).max() < 1e-12 * np.abs(f).sum()                      # moment balance
    Kmax = np.abs(out["K"]).max()
    for c in range(3):
        t = np.zeros_like(u).reshape(-1, 3)
        t[:, c] = 1.0
        assert np.abs(K @ t.ravel()).max() < 1e-11 * Kmax                   # rigid translation
    Wm = np.array([[0, -0.3, 0.2], [0.3, 0, -0.7], [-0.2, 0.7, 0]])
    rotv = (xc @ Wm.T).ravel()
    assert np.abs(K @ rotv - (f @ Wm.T).ravel()).max() < 1e-10 * scale      # infinitesimal rotation
    assert abs(K - K.T).max() < 1e-12 * Kmax                                # symmetric


def test_patch_test_interior_nodes_unloaded():
    """Affine displacement on the fully populated lower half of the C0 mesh gives a uniform
    stress, and interior nodes receive no net internal force."""
    w = W.get("c0")
    m, ps = setup(w)
    s = W.make_state(w, ps)
    nd = m.nodes()
    X = node_xyz(w, nd)
    A = np.array([[1e-3, 2e-4, -3e-4], [5e-4, -2e-3, 1e-4], [-1e-4, 3e-4, 4e-3]])
    u = (X @ A.T).ravel()
    out = m.assemble(s, u, want_K=False)
    sig = out["sigma"]
    assert np.abs(sig - sig[:, :1]).max() < 1e-10 * np.abs(sig).max()
    f = out["f_int"].reshape(-1, 3)
    interior = (nd[:, 0] > 0) & (nd[:, 0] < 8) & (nd[:, 1] > 0) & (nd[:, 1] < 8) & (nd[:, 2] > 0) & (nd[:, 2] < 4)
    assert interior.sum() == 7 * 7 * 3
    assert np.abs(f[interior]).max() < 1e-12 * np.abs(f).max()


@pytest.mark.parametrize("kind,jit", [("sphere", None), ("cone", 1)])
def test_external_force_total(kind, jit):
    from oracle.oracle import residual
    w, m, ps, s, u = _problem(kind, jit, math.inf)
    fe = m.external_force(s).reshape(-1, 3)
    g = np.array([0.0, 0.0, -9.81])
    assert np.abs(fe.sum(axis=0) - g * s["mass"].sum()).max() < 1e-13 * np.abs(g).max() * s["mass"].sum()
    fi = m.assemble(s, u, want_K=False)["f_int"]
    d = W.dirichlet_dofs(m.nodes())
    r, rn = residual(fi, fe.ravel(), d)
    ref = np.where(d == 1, 0.0, fi - fe.ravel())
    assert np.array_equal(r, ref)
    assert abs(rn - np.sqrt(np.sum(ref * ref))) < 1e-15 * rn


@pytest.mark.parametrize("kind,jit,sy", CASES)
def test_committed_state(kind, jit, sy):
    """The history the assembly commits (Section 2.1, updated Lagrangian; Section 2.2):
    F_new = dF F_n with dF = I + sum_v u_v (x) grad S_v rebuilt here from the basis; b_e is the
    trial tensor dF b_n dF^T at elastic points; and a step from the committed state (b_n = b_e,
    J_n = J, F_n = F_new) with no further displacement returns the same Cauchy stress."""
    w, m, ps, s, u = _problem(kind, jit, sy)
    out = m.assemble(s, u, want_K=False)
    U = u.reshape(-1, 3)
    n = ps.n
    Jnew = np.zeros(n)
    for p in range(n):
        nd, S, dS = m.point_basis(ps.x[:, p], ps.l[:, p])
        dF = np.eye(3) + U[nd].T @ dS
        Fn = s["Fn"][:, p].reshape(3, 3)
        Fp = out["Fnew"][:, p].reshape(3, 3)
        assert np.abs(Fp - dF @ Fn).max() < 1e-14
        Jnew[p] = np.linalg.det(dF) * s["Jn"][p]
        if not out["plastic"][p]:
            bn = s["bn"][:, p]
            B = dF @ np.array([[bn[0], bn[3], bn[5]], [bn[3], bn[1], bn[4]], [bn[5], bn[4], bn[2]]]) @ dF.T
            be = out["be"][:, p]
            assert np.abs(be - B[[0, 1, 2, 0, 1, 0], [0, 1, 2, 1, 2, 2]]).max() < 1e-14
    assert np.abs(Jnew / np.array([np.linalg.det(out["Fnew"][:, p].reshape(3, 3)) for p in range(n)]) - 1).max() < 1e-13
    s2 = dict(s, bn=out["be"], Jn=Jnew, Fn=out["Fnew"])
    again = m.assemble(s2, np.zeros_like(u), want_K=False)
    assert np.abs(again["sigma"] - out["sigma"]).max() < 1e-12 * np.abs(out["sigma"]).max()


def test_trial_stress_output():
    """q_trial is the von Mises stress sqrt(3 J2) of the trial Kirchhoff stress: with no yield
    limit it equals that of the returned stress (tau = J sigma); with a finite limit a point
    is plastic exactly where q_trial exceeds it. The 70th percentile of q_trial as the limit
    (the rule that sets the partial-yielding workload's yield stress) yields 30 % of them."""
    w, m, ps, s, u = _problem("sphere", 0, math.inf)
    el = m.assemble(s, u, want_K=False)
    J = np.array([np.linalg.det(el["Fnew"][:, p].reshape(3, 3)) for p in range(ps.n)])
    tau = el["sigma"] * J
    dev = tau.copy()
    dev[:3] -= tau[:3].mean(axis=0)
    q = np.sqrt(1.5 * (dev[0] ** 2 + dev[1] ** 2 + dev[2] ** 2 + 2 * (dev[3] ** 2 + dev[4] ** 2 + dev[5] ** 2)))
    assert np.abs(el["q_trial"] - q).max() < 1e-12 * q.max()
    sy = float(np.percentile(el["q_trial"], 70))
    pl = m.assemble(dict(s, sy=np.full(ps.n, sy)), u, want_K=False)
    assert np.array_equal(pl["plastic"].astype(bool), el["q_trial"] > sy)
    assert abs(pl["plastic"].mean() - 0.3) < 2.0 / ps.n
    assert np.array_equal(pl["q_trial"], el["q_trial"])


def test_partial_yield_workload_sigma_y():
    """The partial-yielding sphere workload's yield stress is the stored output of its
    oracle-only script, and the oracle yields 30 % of its points at that stress."""
    import json
    from pathlib import Path
    rec = json.loads((Path(__file__).resolve().parent / "golden" / "c1b_sigma_y.json").read_text())
    w = W.get("c1b")
    assert w.sy == rec["sigma_y"]
    from tests.golden.make_c1b_sigma_y import trial_q
    q = trial_q(W.get("c1"))
    assert float(np.percentile(q, 70)) == rec["sigma_y"]
    assert abs(np.mean(q > w.sy) - 0.3) < 1e-4


@pytest.mark.parametrize("kind,jit,sy", [("sphere", 0, 40.0), ("box", None, math.inf)])
def test_threaded_timing_driver(kind, jit, sy):
    """The all-cores timing mode adds the same per-point shares: one thread reproduces the
    serial assembly bit for bit, several threads agree to rounding, stress identical."""
    w, m, ps, s, u = _problem(kind, jit, sy)
    ref = m.assemble(s, u)
    one = m.assemble_threads(s, u, 1)
    assert np.array_equal(one["f_int"], ref["f_int"]) and np.array_equal(one["K"], ref["K"])
    assert np.array_equal(one["sigma"], ref["sigma"])
    for t in (3, 8):
        par = m.assemble_threads(s, u, t)
        assert np.abs(par["f_int"] - ref["f_int"]).max() <= 1e-14 * np.abs(ref["f_int"]).max()
        assert np.abs(par["K"] - ref["K"]).max() <= 1e-14 * np.abs(ref["K"]).max()
        assert np.array_equal(par["sigma"], ref["sigma"])
        again = m.assemble_threads(s, u, t)
        assert np.array_equal(again["f_int"], par["f_int"]) and np.array_equal(again["K"], par["K"])
