"""Pins of the oracle's GIMP basis (Section 3.2) against properties and closed forms that
do not depend on how the oracle integrates: partition of unity, linear completeness, the
1D cpGIMP closed form on a uniform mesh, Gauss quadrature of the convolution, central
differences, and C1 continuity across a hanging-node interface."""
import numpy as np
import pytest

import workloads as W
from oracle.oracle import OracleMesh
from tests.helpers import leaf_sizes, node_xyz, setup, tiny_workload


def _basis_all(m, ps, idx):
    for p in idx:
        yield p, m.point_basis(ps.x[:, p], ps.l[:, p])


@pytest.mark.parametrize("kind,jit", [("sphere", None), ("sphere", 0), ("cone", 1), ("box", 3)])
def test_partition_of_unity_and_linear_completeness(kind, jit):
    w = tiny_workload(kind)
    m, ps = setup(w, jitter=jit)
    X = node_xyz(w, m.nodes())
    for p, (nd, S, dS) in _basis_all(m, ps, range(ps.n)):
        assert abs(S.sum() - 1.0) < 1e-14
        assert np.abs(dS.sum(axis=0)).max() < 1e-11
        assert np.abs(S @ X[nd] - ps.x[:, p]).max() < 1e-14
        assert np.abs(X[nd].T @ dS - np.eye(3)).max() < 1e-12


def test_partition_of_unity_c1_sample():
    w = W.get("c1")
    m, ps = setup(w)
    X = node_xyz(w, m.nodes())
    rng = np.random.default_rng(0)
    for p, (nd, S, dS) in _basis_all(m, ps, rng.choice(ps.n, 3000, replace=False)):
        assert abs(S.sum() - 1.0) < 1e-14
        assert np.abs(dS.sum(axis=0)).max() < 1e-10
        assert np.abs(X[nd].T @ dS - np.eye(3)).max() < 1e-12


def _s1(d, h, l):
    a = np.abs(d)
    return np.where(a < l, 1 - (d * d + l * l) / (2 * h * l),
                    np.where(a < h - l, 1 - a / h, np.where(a < h + l, (h + l - a) ** 2 / (4 * h * l), 0.0)))


def _ds1(d, h, l):
    a, s = np.abs(d), np.sign(d)
    return np.where(a < l, -d / (h * l),
                    np.where(a < h - l, -s / h, np.where(a < h + l, -s * (h + l - a) / (2 * h * l), 0.0)))


def test_uniform_mesh_closed_form():
    """On a uniform mesh the GIMP weight is the tensor product of the 1D convolution of a
    hat function of half-width h with a box of half-width l (l <= h/2)."""
    w = W.get("c0")
    m = OracleMesh(w.crit())
    X = node_xyz(w, m.nodes())
    h = w.h0
    rng = np.random.default_rng(5)
    for _ in range(400):
        x = rng.uniform(0.15, 0.85, 3)
        l = rng.uniform(0.1 * h, 0.5 * h, 3)
        nd, S, dS = m.point_basis(x, l)
        d = x[None, :] - X
        f = _s1(d, h, l[None, :])
        g = _ds1(d, h, l[None, :])
        Sx = f.prod(axis=1)
        dSx = np.stack([g[:, 0] * f[:, 1] * f[:, 2], f[:, 0] * g[:, 1] * f[:, 2], f[:, 0] * f[:, 1] * g[:, 2]], 1)
        exp_nodes = set(np.nonzero(Sx > 0)[0]) | set(np.nonzero(np.abs(dSx).sum(1) > 0)[0])
        assert exp_nodes <= set(nd.tolist())
        assert np.abs(S - Sx[nd]).max() < 1e-14
        assert np.abs(dS - dSx[nd]).max() < 1e-12
        mask = np.ones(X.shape[0], bool)
        mask[nd] = False
        assert np.abs(Sx[mask]).max(initial=0) == 0


def _phi_tilde(m, w, lv, s, cells, e, P):
    """phi~ of leaf e at points P (3, q): C_K^T times the 8 trilinear vertex functions."""
    n, ids, cm = cells
    lo = lv[e, :3] * w.h_min
    h = s[e] * w.h_min
    xi = (P - lo[:, None]) / h
    phi = np.stack([np.prod([xi[a] if (v >> a) & 1 else 1 - xi[a] for a in range(3)], axis=0) for v in range(8)])
    return ids[e, :n[e]], cm[e, :, :n[e]].T @ phi


@pytest.mark.parametrize("kind,jit", [("sphere", 0), ("cone", 2)])
def test_gauss_quadrature_of_convolution(kind, jit):
    """4x4x4 Gauss-Legendre quadrature of (1/V_p) int_{Omega_p cap K} phi~ over every
    overlapped leaf reproduces S_vp (the one-point rule of the method is exact for
    trilinear functions; so is the oracle's antiderivative evaluation)."""
    w = tiny_workload(kind)
    m, ps = setup(w, jitter=jit)
    lv = m.leaves()
    s = leaf_sizes(w, lv)
    cells = m.cells()
    gx, gw = np.polynomial.legendre.leggauss(4)
    lo_all = lv[:, :3] * w.h_min
    hi_all = lo_all + (s * w.h_min)[:, None]
    for p in range(0, ps.n, 3):
        x, l = ps.x[:, p], ps.l[:, p]
        a0 = np.maximum(x - l, lo_all)
        a1 = np.minimum(x + l, hi_all)
        ov = a1 - a0
        hit = np.nonzero(np.all(ov > 1e-12 * 2 * l, axis=1))[0]
        acc = {}
        for e in hit:
            pts = [(a0[e, a] + a1[e, a]) / 2 + (a1[e, a] - a0[e, a]) / 2 * gx for a in range(3)]
            wts = [(a1[e, a] - a0[e, a]) / 2 * gw for a in range(3)]
            Z, Y, Xg = np.meshgrid(pts[2], pts[1], pts[0], indexing="ij")
            WZ, WY, WX = np.meshgrid(wts[2], wts[1], wts[0], indexing="ij")
            P = np.stack([Xg.ravel(), Y.ravel(), Z.ravel()])
            wq = (WX * WY * WZ).ravel()
            ids, ph = _phi_tilde(m, w, lv, s, cells, e, P)
            for i, node in enumerate(ids):
                acc[int(node)] = acc.get(int(node), 0.0) + ph[i] @ wq / np.prod(2 * l)
        nd, S, dS = m.point_basis(x, l)
        for i, node in enumerate(nd):
            assert abs(S[i] - acc.get(int(node), 0.0)) < 1e-14


@pytest.mark.parametrize("kind,jit", [("sphere", 0), ("box", 1)])
def test_gradient_is_position_derivative(kind, jit):
    w = tiny_workload(kind)
    m, ps = setup(w, jitter=jit)
    hstep = 1e-6 * w.h_min
    for p in range(0, ps.n, 5):
        x, l = ps.x[:, p], ps.l[:, p]
        if np.any(x - l < 2 * hstep) or np.any(x + l > np.array(w.base) * w.h0 - 2 * hstep):
            continue
        nd, S, dS = m.point_basis(x, l)
        for a in range(3):
            e = np.zeros(3)
            e[a] = hstep
            n1, S1, _ = m.point_basis(x + e, l)
            n0, S0, _ = m.point_basis(x - e, l)
            d1 = dict(zip(n1.tolist(), S1))
            d0 = dict(zip(n0.tolist(), S0))
            fd = np.array([(d1.get(k, 0.0) - d0.get(k, 0.0)) / (2 * hstep) for k in nd.tolist()])
            assert np.abs(fd - dS[:, a]).max() < 1e-6 * np.abs(dS).max()


def test_c1_continuity_across_hanging_interface():
    """Sweep a GIMP (half side 0.5 h_fine) along a line crossing a coarse/fine interface with
    hanging nodes: S and grad S are continuous, i.e. their increments shrink in proportion
    to the step (a jump would not shrink)."""
    w = tiny_workload("sphere", lvl_extra=2)
    m = OracleMesh(w.crit())
    ijk, sup, wts, own = m.hanging()
    assert len(ijk) > 0
    hx = node_xyz(w, ijk[len(ijk) // 2])
    lv = m.leaves()
    lvl = lv[own[len(ijk) // 2], 3]
    hc = w.h_min * (1 << (w.lvl_max - lvl))
    l = np.full(3, 0.25 * hc)
    path0 = hx + np.array([-0.9 * hc, 0.37 * hc, 0.21 * hc])
    path1 = hx + np.array([0.9 * hc, -0.31 * hc, 0.17 * hc])

    def sweep(nsteps):
        ts = np.linspace(0, 1, nsteps)
        allS = []
        for t in ts:
            x = path0 + t * (path1 - path0)
            x = np.clip(x, l + 1e-9, np.array(w.base) * w.h0 - l - 1e-9)
            nd, S, dS = m.point_basis(x, l)
            allS.append({int(k): (S[i], dS[i]) for i, k in enumerate(nd)})
        keys = set().union(*[set(d) for d in allS])
        jumpS = jumpG = 0.0
        for a, b in zip(allS[:-1], allS[1:]):
            for k in keys:
                sa, ga = a.get(k, (0.0, np.zeros(3)))
                sb, gb = b.get(k, (0.0, np.zeros(3)))
                jumpS = max(jumpS, abs(sb - sa))
                jumpG = max(jumpG, np.abs(gb - ga).max())
        return jumpS, jumpG

    jS1, jG1 = sweep(201)
    jS2, jG2 = sweep(801)
    assert jS1 / jS2 > 3.0 and jG1 / jG2 > 3.0
