"""Pins of the oracle's Hencky / von Mises update and consistent tangent (Section 2.2):
rigid rotation, objectivity, the uniaxial closed forms (elastic: Section 6.2 stress
solution E (l0/l) ln(l/l0) for nu = 0), consistency on the yield surface, the tangent
against central differences, and small-strain elasticity at the undeformed state."""
import math

import numpy as np
import pytest

from oracle.oracle import material_point

RNG = np.random.default_rng(42)


def rot(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q @ np.diag(np.sign(np.diag(r)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def sym6(A):
    return np.array([A[0, 0], A[1, 1], A[2, 2], A[0, 1], A[1, 2], A[0, 2]])


def full(v):
    return np.array([[v[0], v[3], v[5]], [v[3], v[1], v[4]], [v[5], v[4], v[2]]])


def rand_state(rng, amp=0.05):
    Fn = np.eye(3) + rng.normal(0, amp, (3, 3))
    while np.linalg.det(Fn) <= 0:
        Fn = np.eye(3) + rng.normal(0, amp, (3, 3))
    dF = np.eye(3) + rng.normal(0, amp, (3, 3))
    return dF, sym6(Fn @ Fn.T), np.linalg.det(Fn)


def test_rigid_rotation_is_stress_free():
    for _ in range(50):
        R = rot(RNG)
        o = material_point(R, sym6(np.eye(3)), 1.0, 1e5, 0.3, 50.0)
        assert np.abs(o["sigma"]).max() < 1e-10 * 1e5 * 1e-3


@pytest.mark.parametrize("sy", [math.inf, 30.0])
def test_objectivity(sy):
    for _ in range(50):
        dF, bn, Jn = rand_state(RNG)
        Q = rot(RNG)
        a = material_point(dF, bn, Jn, 1e4, 0.3, sy)
        b = material_point(Q @ dF, bn, Jn, 1e4, 0.3, sy)
        Sa, Sb = full(a["sigma"]), full(b["sigma"])
        assert np.abs(Q @ Sa @ Q.T - Sb).max() < 1e-12 * np.abs(Sa).max()
        assert a["plastic"] == b["plastic"]


@pytest.mark.parametrize("lam", [0.6, 0.8, 0.95, 1.05, 1.3])
def test_uniaxial_elastic_closed_form(lam):
    E = 1e6
    o = material_point(np.diag([1.0, 1.0, lam]), sym6(np.eye(3)), 1.0, E, 0.0, math.inf)
    # column compressed from length l0 to l: sigma_z = E (l0/l) ln(l/l0)
    assert abs(o["sigma"][2] - E / lam * math.log(lam)) < 1e-12 * E
    assert np.abs(o["sigma"][[0, 1, 3, 4, 5]]).max() < 1e-12 * E
    nu = 0.3
    lamL, G = E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))
    o = material_point(np.diag([1.0, 1.0, lam]), sym6(np.eye(3)), 1.0, E, nu, math.inf)
    assert abs(o["sigma"][2] - (lamL + 2 * G) * math.log(lam) / lam) < 1e-12 * E
    assert abs(o["sigma"][0] - lamL * math.log(lam) / lam) < 1e-12 * E


@pytest.mark.parametrize("lam", [0.7, 0.9, 0.99])
def test_uniaxial_plastic_closed_form(lam):
    E, nu, sy = 1e5, 0.3, 50.0
    G, Kb = E / (2 * (1 + nu)), E / (3 * (1 - 2 * nu))
    assert 2 * G * abs(math.log(lam)) > sy
    o = material_point(np.diag([1.0, 1.0, lam]), sym6(np.eye(3)), 1.0, E, nu, sy)
    e = math.log(lam)
    assert o["plastic"]
    assert abs(o["sigma"][2] - (Kb * e - 2.0 / 3.0 * sy) / lam) < 1e-12 * E
    assert abs(o["sigma"][0] - (Kb * e + 1.0 / 3.0 * sy) / lam) < 1e-12 * E


def test_plastic_points_on_yield_surface():
    n = 0
    for _ in range(200):
        dF, bn, Jn = rand_state(RNG, 0.05)
        o = material_point(dF, bn, Jn, 2e5, 0.3, 100.0)
        if not o["plastic"]:
            continue
        n += 1
        tau = full(o["tau"])
        s = tau - np.trace(tau) / 3 * np.eye(3)
        assert abs(math.sqrt(1.5 * np.sum(s * s)) - 100.0) < 1e-12 * 2e5
    assert n > 100


def _phi(dF, bn, Jn, E, nu, sy):
    o = material_point(dF, bn, Jn, E, nu, sy, want_tangent=False)
    return full(o["tau"]) @ np.linalg.inv(dF).T, o["plastic"]


@pytest.mark.parametrize("sy", [math.inf, 100.0])
def test_tangent_matches_central_differences(sy):
    """a:Z = (1/J) d/de [tau((I+eZ)dF) ((I+eZ)dF)^-T] dF^T, the variation of the nodal force
    with the displacement gradient (Z = grad_x du)."""
    checked = 0
    for _ in range(60):
        dF, bn, Jn = rand_state(RNG, 0.05)
        o = material_point(dF, bn, Jn, 2e5, 0.3, sy)
        if np.isfinite(sy) and abs(o["q_trial"] - sy) < 1e-3 * sy:
            continue
        a = o["a"].reshape(9, 9)
        J = o["J"]
        for _ in range(3):
            Z = RNG.normal(size=(3, 3))
            h = 1e-6
            p, pl1 = _phi((np.eye(3) + h * Z) @ dF, bn, Jn, 2e5, 0.3, sy)
            m, pl0 = _phi((np.eye(3) - h * Z) @ dF, bn, Jn, 2e5, 0.3, sy)
            if pl1 != pl0 or pl1 != o["plastic"]:
                continue
            fd = (p - m) / (2 * h) @ dF.T / J
            an = (a @ Z.reshape(9)).reshape(3, 3)
            assert np.abs(fd - an).max() < 1e-6 * np.abs(an).max()
            checked += 1
    assert checked > 100


def test_undeformed_tangent_is_small_strain_elasticity():
    E, nu = 1e4, 0.3
    lamL, G = E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))
    o = material_point(np.eye(3), sym6(np.eye(3)), 1.0, E, nu, math.inf)
    d = np.eye(3)
    C = lamL * np.einsum("ij,kl->ijkl", d, d) + G * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d))
    assert np.abs(o["a"] - C).max() < 1e-12 * E
    assert np.abs(o["sigma"]).max() == 0.0


# ---------------------------------------------------------------- committed elastic strain
# The updated-Lagrangian scheme (Section 2.1) carries the elastic left Cauchy-Green tensor
# b_e and F to the next step; with Hencky elasticity and a perfectly plastic von Mises surface
# (Section 2.2) the committed b_e is fixed by three facts that do not depend on how the return
# is coded: an elastic step commits the trial tensor dF b_n dF^T itself; a plastic step keeps
# the principal directions of the trial tensor and its volume (the radial return changes only
# the deviatoric strain, so det b_e = det b_tr); and the Hencky stress of the committed b_e is
# the returned stress, which lies on the yield surface.

def _btr(dF, bn):
    return dF @ full(bn) @ dF.T


def _hencky_tau(b, E, nu):
    """Kirchhoff stress of Hencky elasticity at the elastic left Cauchy-Green tensor b:
    tau = lam tr(eps) I + 2 G eps with eps = log(b) / 2 (numpy eigendecomposition)."""
    lam, G = E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))
    w, V = np.linalg.eigh(b)
    eps = 0.5 * (V * np.log(w)) @ V.T
    return lam * np.trace(eps) * np.eye(3) + 2 * G * eps


def test_committed_be_elastic_is_trial():
    for _ in range(50):
        dF, bn, Jn = rand_state(RNG)
        o = material_point(dF, bn, Jn, 1e4, 0.3, math.inf, want_tangent=False)
        B = _btr(dF, bn)
        assert not o["plastic"]
        assert np.abs(full(o["be"]) - B).max() < 1e-14 * np.abs(B).max() * 10
        assert np.abs(_hencky_tau(full(o["be"]), 1e4, 0.3) - full(o["tau"])).max() < 1e-11 * 1e4 * 0.05


def test_committed_be_plastic_coaxial_volume_and_stress():
    E, nu, sy = 2e5, 0.3, 100.0
    n = 0
    for _ in range(200):
        dF, bn, Jn = rand_state(RNG, 0.05)
        o = material_point(dF, bn, Jn, E, nu, sy, want_tangent=False)
        if not o["plastic"]:
            continue
        n += 1
        B, be, tau = _btr(dF, bn), full(o["be"]), full(o["tau"])
        # coaxial with the trial tensor: the two commute
        assert np.abs(be @ B - B @ be).max() < 1e-13 * np.abs(B).max() ** 2
        # the radial return keeps the volumetric strain
        assert abs(np.linalg.det(be) / np.linalg.det(B) - 1.0) < 1e-13
        # the committed tensor's Hencky stress is the returned stress, on the yield surface
        th = _hencky_tau(be, E, nu)
        assert np.abs(th - tau).max() < 1e-12 * E
        s = th - np.trace(th) / 3 * np.eye(3)
        assert abs(math.sqrt(1.5 * np.sum(s * s)) - sy) < 1e-12 * E
    assert n > 100


@pytest.mark.parametrize("sy", [math.inf, 100.0])
def test_recommitted_state_reproduces_stress(sy):
    """A new step from the committed state with no further displacement (dF = I,
    b_n = b_e, J_n = J) returns the committed stress: the committed state is a fixed point."""
    E, nu = 2e5, 0.3
    for _ in range(60):
        dF, bn, Jn = rand_state(RNG, 0.05)
        o = material_point(dF, bn, Jn, E, nu, sy, want_tangent=False)
        r = material_point(np.eye(3), o["be"], o["J"], E, nu, sy, want_tangent=False)
        assert np.abs(r["tau"] - o["tau"]).max() < 1e-11 * E
        assert np.abs(r["sigma"] - o["sigma"]).max() < 1e-11 * E
        assert abs(r["J"] - o["J"]) < 1e-15
