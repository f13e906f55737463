"""Pins of the oracle's adjoint gradients of L = lambda . f_int(u) with respect to the
per-point parameters (E, nu, sigma_y, V_n): central finite differences of the forward
assembly, and Euler-homogeneity identities of the stress in the parameters."""
import math

import numpy as np
import pytest

import workloads as W
from tests.helpers import setup, tiny_workload


def _prob(jit, sy):
    w = tiny_workload("sphere", E=1e4, nu=0.3, sy=sy, Fn_std=0.03)
    m, ps = setup(w, jitter=jit)
    s = W.make_state(w, ps)
    nd = m.nodes()
    u = W.make_u(w, nd, amp=2e-3)
    lam = W.make_lambda(w, nd)
    return w, m, ps, s, u, lam


@pytest.mark.parametrize("jit,sy", [(None, math.inf), (0, 20.0), (1, 60.0)])
def test_adjoint_matches_central_differences(jit, sy):
    w, m, ps, s, u, lam = _prob(jit, sy)
    g = m.adjoint(s, u, lam)
    rng = np.random.default_rng(3)
    plastic = m.assemble(s, u, want_K=False)["plastic"]
    for p in rng.choice(ps.n, 12, replace=False):
        for key, grad in (("E", "dE"), ("nu", "dnu"), ("sy", "dsy"), ("vol", "dV")):
            if key == "sy" and not math.isfinite(s["sy"][p]):
                assert g["dsy"][p] == 0.0
                continue
            h = 1e-5 * abs(s[key][p])  # L sums all points: a smaller step is roundoff-limited
            vals = []
            for sgn in (1, -1):
                s2 = dict(s)
                s2[key] = s[key].copy()
                s2[key][p] += sgn * h
                o = m.assemble(s2, u, want_K=False)
                assert o["plastic"][p] == plastic[p]
                vals.append(lam @ o["f_int"])
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - g[grad][p]) <= 1e-6 * max(abs(fd), 1e-8 * abs(lam @ m.assemble(s, u, False)["f_int"]) / ps.n)


@pytest.mark.parametrize("jit,sy", [(None, math.inf), (0, 20.0), (2, 60.0)])
def test_euler_homogeneity(jit, sy):
    """tau is homogeneous of degree one in (E) for elastic points and in (E, sigma_y) for
    plastic points, and L is linear in every V_n."""
    w, m, ps, s, u, lam = _prob(jit, sy)
    g = m.adjoint(s, u, lam)
    o = m.assemble(s, u, want_K=False)
    L = lam @ o["f_int"]
    Lp = s["vol"] * g["dV"]
    assert abs(Lp.sum() - L) < 1e-12 * np.abs(Lp).sum()
    el = o["plastic"] == 0
    scale = np.abs(Lp).max()
    assert np.abs(s["E"][el] * g["dE"][el] - Lp[el]).max(initial=0) < 1e-12 * scale
    assert np.all(g["dsy"][el] == 0.0)
    pl = ~el
    if math.isfinite(sy):
        assert pl.sum() > 0
        r = s["E"][pl] * g["dE"][pl] + s["sy"][pl] * g["dsy"][pl] - Lp[pl]
        assert np.abs(r).max(initial=0) < 1e-12 * scale
