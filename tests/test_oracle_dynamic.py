"""Pins of the oracle's inertia term (weak form of Section 2.1 with Newmark's method at
gamma = 1, beta = 1/2, Section 2.4): its tangent against differences of the force, the
consistent mass (symmetric, positive semi-definite, rows summing to the lumped mass given by
the body-force term), constant-acceleration kinematics that the scheme integrates exactly
(free fall), and the velocity-only case."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from tests.helpers import setup, tiny_workload

DT = 1e-3


def _problem(kind, jit):
    w = tiny_workload(kind, E=1e4, nu=0.3, sy=math.inf)
    m, ps = setup(w, jitter=jit)
    s = W.make_state(w, ps)
    vel = W.make_velocity(w, ps)
    u = W.make_u(w, m.nodes(), amp=1e-4)
    return w, m, ps, s, vel, u


def _K(m, K):
    rp, col = m.csr()
    n = 3 * m.counts()["n_node"]
    return sp.csr_matrix((K, col, rp), shape=(n, n))


CASES = [("sphere", None), ("cone", 1), ("box", 2)]


@pytest.mark.parametrize("kind,jit", CASES)
def test_inertia_tangent_is_jacobian(kind, jit):
    w, m, ps, s, vel, u = _problem(kind, jit)
    out = m.inertia(s, u, vel, DT)
    K = _K(m, out["K_mass"])
    rng = np.random.default_rng(2)
    for _ in range(3):
        d = rng.normal(size=u.size)
        h = 1e-6
        fp = m.inertia(s, u + h * d, vel, DT, want_K=False)["f_iner"]
        fm = m.inertia(s, u - h * d, vel, DT, want_K=False)["f_iner"]
        kd = K @ d
        assert np.abs((fp - fm) / (2 * h) - kd).max() < 1e-9 * np.abs(kd).max()


@pytest.mark.parametrize("kind,jit", CASES)
def test_consistent_mass_properties(kind, jit):
    w, m, ps, s, vel, u = _problem(kind, jit)
    K = _K(m, m.inertia(s, u, vel, DT)["K_mass"])
    M = K * (DT * DT / 2.0)
    assert abs(M - M.T).max() <= 1e-15 * abs(M).max()
    rng = np.random.default_rng(3)
    for _ in range(5):
        d = rng.normal(size=u.size)
        assert d @ (M @ d) >= -1e-14 * np.abs(M).max() * d @ d
    # rows sum to the lumped mass sum_p S_vp m_p, which the body-force term gives for g = (1,1,1)
    lumped = m.external_force(dict(s, g=(1.0, 1.0, 1.0)))
    assert np.abs(M @ np.ones(u.size) - lumped).max() <= 1e-13 * np.abs(lumped).max()
    # total mass: one component of the uniform field carries every point's mass once
    assert abs(lumped[0::3].sum() - s["mass"].sum()) <= 1e-12 * s["mass"].sum()


@pytest.mark.parametrize("kind,jit", CASES)
def test_free_fall_is_integrated_exactly(kind, jit):
    """A rigid translation u = v0 dt + g dt^2 / 2 of points moving with v0 has acceleration g
    (Newmark with beta = 1/2 is exact for constant acceleration): the inertia force equals the
    body force, a_p = g and v_p,new = v0 + g dt at every point."""
    w, m, ps, s, vel, u = _problem(kind, jit)
    g = np.array([0.3, -0.2, -9.81])
    v0 = np.array([0.5, 0.1, -0.7])
    vel = np.tile(v0[:, None], (1, ps.n))
    u = np.tile(v0 * DT + 0.5 * g * DT * DT, m.counts()["n_node"])
    out = m.inertia(s, u, vel, DT, want_K=False)
    fe = m.external_force(dict(s, g=tuple(g)))
    assert np.abs(out["f_iner"] - fe).max() <= 1e-9 * np.abs(fe).max()
    assert np.abs(out["a"] - g[:, None]).max() <= 1e-9 * np.abs(g).max()
    assert np.abs(out["v"] - (v0 + g * DT)[:, None]).max() <= 1e-12


@pytest.mark.parametrize("kind,jit", CASES)
def test_velocity_only_and_totals(kind, jit):
    w, m, ps, s, vel, u = _problem(kind, jit)
    zero = np.zeros_like(u)
    out = m.inertia(s, zero, vel, DT, want_K=False)
    # u = 0: a_p = -2 v_p / dt, and the nodal forces sum to sum_p m_p a_p per component
    assert np.abs(out["a"] + 2.0 * vel / DT).max() <= 1e-12 * np.abs(vel).max() / DT
    tot = out["f_iner"].reshape(-1, 3).sum(axis=0)
    ref = (s["mass"][None, :] * out["a"]).sum(axis=1)
    assert np.abs(tot - ref).max() <= 1e-12 * np.abs(ref).max()
    out0 = m.inertia(s, zero, np.zeros_like(vel), DT, want_K=False)
    assert np.abs(out0["f_iner"]).max() == 0.0
