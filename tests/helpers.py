"""Shared test helpers: small meshes and seeded inputs (no method arithmetic here)."""
from __future__ import annotations

import math

import numpy as np

import workloads as W
from workloads.configs import BODY_BOX, BODY_CONE, BODY_NONE, BODY_SPHERE, Workload


def tiny_workload(kind: str = "sphere", lvl_extra: int = 2, E=1e3, nu=0.3, sy=math.inf, Fn_std=0.0,
                  base=(3, 3, 3), ppa=2) -> Workload:
    """A few-hundred-point mesh with hanging nodes (sphere/cone/box near a corner). ppa is the
    number of points per axis in a leaf, or a function of the leaf level."""
    if kind == "sphere":
        bk, body, dx = BODY_SPHERE, (0.55, 0.45, 0.6, 0.12), 0.08
    elif kind == "cone":
        bk, body, dx = BODY_CONE, (0.5, 0.5, 0.55, 0.1, math.tan(math.radians(30)), 1.0), 0.05
    elif kind == "box":
        bk, body, dx = BODY_BOX, (0.6, 0.8, 0.3, 0.45, 0.7, 1.0), 0.06
    else:
        bk, body, dx = BODY_NONE, (), 0.0
    ppa_fn = ppa if callable(ppa) else (lambda lv: ppa)
    return Workload(name=f"tiny_{kind}", lo=(0.0, 0.0, 0.0), base=base, h0=1.0 / base[0], lvl_base=2,
                    lvl_max=2 + lvl_extra, body_kind=bk, body=body, dx_region=dx, ppa=ppa_fn,
                    E=E, nu=nu, sy=sy, Fn_std=Fn_std, seed_state=7, seed_u=8, seed_lambda=9,
                    drop_inside_body=True)


def morton3_np(x, y, z):
    """Morton key by bit interleaving (x -> bit 3b, y -> 3b+1, z -> 3b+2), vectorised."""
    x = np.asarray(x, np.uint64); y = np.asarray(y, np.uint64); z = np.asarray(z, np.uint64)
    k = np.zeros(np.broadcast(x, y, z).shape, np.uint64)
    for b in range(21):
        bb = np.uint64(b)
        k |= ((x >> bb) & np.uint64(1)) << np.uint64(3 * b)
        k |= ((y >> bb) & np.uint64(1)) << np.uint64(3 * b + 1)
        k |= ((z >> bb) & np.uint64(1)) << np.uint64(3 * b + 2)
    return k


def leaf_sizes(w: Workload, lv):
    return (1 << (w.lvl_max - lv[:, 3])).astype(np.int64)


def setup(w: Workload, jitter: int | None = None, shuffle_seed=12345):
    from oracle.oracle import OracleMesh
    m = OracleMesh(w.crit())
    lv = m.leaves()
    ps = W.make_points(w, lv[:, :3], lv[:, 3], shuffle_seed=shuffle_seed)
    if jitter is not None:
        ps = W.jitter_points(w, ps, jitter)
    m.set_points(ps.x, ps.l)
    return m, ps


def node_xyz(w: Workload, ijk):
    return np.asarray(w.lo)[None, :] + np.asarray(ijk, np.float64) * w.h_min
