"""Seeded input generators (numpy only).

Points are placed on a given leaf set (anchor lattice coordinates + level), which either
side supplies from its own octree; the leaf sets of the two sides are checked equal before
inputs are shared. Layout of every per-point array is structure-of-arrays with the
component index first: x[c, p].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .configs import BODY_BOX, BODY_CONE, BODY_NONE, BODY_SPHERE, Workload


@dataclass
class PointSet:
    x: np.ndarray      # (3, N) centres
    l: np.ndarray      # (3, N) half side lengths of the GIMP domains

    @property
    def n(self) -> int:
        return int(self.x.shape[1])


def _inside_body(w: Workload, x, y, z):
    b = w.body
    if w.body_kind == BODY_NONE:
        return np.zeros(x.shape, dtype=bool)
    if w.body_kind == BODY_SPHERE:
        return (x - b[0]) ** 2 + (y - b[1]) ** 2 + (z - b[2]) ** 2 <= b[3] ** 2
    if w.body_kind == BODY_CONE:
        rho = np.hypot(x - b[0], y - b[1])
        rad = np.minimum(b[3], (z - b[2]) * b[4])
        return (z >= b[2]) & (z <= b[5]) & (rho <= rad)
    if w.body_kind == BODY_BOX:
        return (x >= b[0]) & (x <= b[1]) & (y >= b[2]) & (y <= b[3]) & (z >= b[4]) & (z <= b[5])
    raise ValueError(w.body_kind)


def make_points(w: Workload, anchors: np.ndarray, levels: np.ndarray, shuffle_seed: int | None = 12345,
                ppa_fn=None) -> PointSet:
    """n x n x n points at the centres of the n^3 sub-boxes of every leaf (n = w.ppa(level)),
    half-length h_K/(2n); points failing w.keep or lying inside the body are dropped. The
    surviving points are shuffled with a seeded permutation so that the point sort has work."""
    anchors = np.asarray(anchors, dtype=np.int64).reshape(-1, 3)
    levels = np.asarray(levels, dtype=np.int64).reshape(-1)
    if "trail_x" in w.extra:
        return _trail_points(w, anchors, levels, shuffle_seed)
    ppa_fn = ppa_fn or w.ppa
    lo = np.asarray(w.lo, dtype=np.float64)
    hmin = w.h_min
    xs, ls = [], []
    ppa = np.array([ppa_fn(int(v)) for v in range(0, w.lvl_max + 1)])
    nleaf = ppa[levels]
    for n in np.unique(nleaf):
        sel = np.nonzero(nleaf == n)[0]
        A = anchors[sel].astype(np.float64)                       # (m, 3)
        h = hmin * np.ldexp(1.0, (w.lvl_max - levels[sel]).astype(np.int64))   # (m,)
        off = (np.arange(n, dtype=np.float64) + 0.5) / n          # (n,)
        iz, iy, ix = np.meshgrid(off, off, off, indexing="ij")
        o = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=0)  # (3, n^3), x fastest
        base = lo[:, None] + A.T * hmin                              # (3, m)
        X = base[:, :, None] + o[:, None, :] * h[None, :, None]      # (3, m, n^3)
        L = np.broadcast_to((h / (2.0 * n))[None, :, None], X.shape)
        xs.append(X.reshape(3, -1))
        ls.append(np.array(L).reshape(3, -1))
    x = np.concatenate(xs, axis=1) if xs else np.zeros((3, 0))
    l = np.concatenate(ls, axis=1) if ls else np.zeros((3, 0))
    keep = np.ones(x.shape[1], dtype=bool)
    if w.keep is not None:
        keep &= w.keep(x[0], x[1], x[2])
    if w.drop_inside_body:
        keep &= ~_inside_body(w, x[0], x[1], x[2])
    x, l = x[:, keep], l[:, keep]
    if shuffle_seed is not None:
        p = np.random.default_rng(shuffle_seed).permutation(x.shape[1])
        x, l = x[:, p], l[:, p]
    return PointSet(np.ascontiguousarray(x), np.ascontiguousarray(l))


def _sub_centres(base, h, n):
    """Centres of the n^3 sub-boxes of boxes with lower corners base (3, m) and sides h (m,):
    (3, m * n^3), sub-box index fastest, x fastest inside it."""
    off = (np.arange(n, dtype=np.float64) + 0.5) / n
    iz, iy, ix = np.meshgrid(off, off, off, indexing="ij")
    o = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=0)
    return (base[:, :, None] + o[:, None, :] * h[None, :, None]).reshape(3, -1)


def _trail_points(w: Workload, anchors, levels, shuffle_seed):
    """Points of a moving-tool workload whose material points are never coarsened: every
    finest-level cell whose centre lies within trail_band of the box swept by the tool over
    trail_x holds trail_ppa^3 points; the rest of the domain holds the usual n^3 points per
    leaf. In a leaf that is only partly covered by the trail, each finest cell outside the
    trail holds one point, so the point domains tile the material exactly."""
    ex = w.extra
    lo = np.asarray(w.lo, dtype=np.float64)
    hmin = w.h_min
    dims = np.asarray(w.lattice_dims(), dtype=np.int64)
    b = w.body
    sw = np.array([ex["trail_x"][0], ex["trail_x"][1] + (b[1] - b[0]), b[2], b[3], b[4], b[5]])
    band, nt = float(ex["trail_band"]), int(ex["trail_ppa"])
    # trail flags on the finest lattice, from the distance of each cell centre to the swept box
    flag = np.zeros(tuple(dims[::-1]), dtype=np.uint8)           # [z, y, x]
    rng_ax = []
    for a in range(3):
        c0 = max(0, int(np.floor((sw[2 * a] - band - lo[a]) / hmin)) - 1)
        c1 = min(int(dims[a]), int(np.ceil((sw[2 * a + 1] + band - lo[a]) / hmin)) + 1)
        rng_ax.append(np.arange(c0, c1))
    cz, cy, cx = np.meshgrid(rng_ax[2], rng_ax[1], rng_ax[0], indexing="ij")
    ctr = [lo[0] + (cx + 0.5) * hmin, lo[1] + (cy + 0.5) * hmin, lo[2] + (cz + 0.5) * hmin]
    d2 = np.zeros(cx.shape)
    for a in range(3):
        da = np.maximum(np.maximum(sw[2 * a] - ctr[a], 0.0), ctr[a] - sw[2 * a + 1])
        d2 += da * da
    tr = d2 <= band * band
    flag[cz[tr], cy[tr], cx[tr]] = 1
    tcells = np.stack([cx[tr], cy[tr], cz[tr]], axis=0)          # (3, n_trail_cells)
    # trail cells per leaf by a summed-volume table
    sat = np.zeros(tuple(dims[::-1] + 1), dtype=np.int32)
    sat[1:, 1:, 1:] = flag.cumsum(0).cumsum(1).cumsum(2)
    side = np.left_shift(1, (w.lvl_max - levels)).astype(np.int64)
    ax, ay, az = anchors[:, 0], anchors[:, 1], anchors[:, 2]
    bx, by, bz = ax + side, ay + side, az + side
    cnt = (sat[bz, by, bx] - sat[az, by, bx] - sat[bz, ay, bx] - sat[bz, by, ax]
           + sat[az, ay, bx] + sat[az, by, ax] + sat[bz, ay, ax] - sat[az, ay, ax])
    xs, ls = [], []
    # leaves without trail cells: n^3 points per leaf
    clean = cnt == 0
    ppa = np.array([w.ppa(int(v)) for v in range(0, w.lvl_max + 1)])
    for n in np.unique(ppa[levels[clean]]):
        sel = np.nonzero(clean & (ppa[levels] == n))[0]
        h = hmin * side[sel].astype(np.float64)
        base = lo[:, None] + anchors[sel].T.astype(np.float64) * hmin
        xs.append(_sub_centres(base, h, int(n)))
        ls.append(np.broadcast_to((h / (2.0 * n))[None, :, None], (3, sel.size, int(n) ** 3)).reshape(3, -1))
    # trail cells: nt^3 points each
    base = lo[:, None] + tcells.astype(np.float64) * hmin
    xs.append(_sub_centres(base, np.full(tcells.shape[1], hmin), nt))
    ls.append(np.full((3, tcells.shape[1] * nt ** 3), hmin / (2.0 * nt)))
    # cells outside the trail inside partly covered leaves: one point each
    for e in np.nonzero((cnt > 0) & (cnt < side ** 3))[0]:
        s = int(side[e])
        sub = flag[az[e]:az[e] + s, ay[e]:ay[e] + s, ax[e]:ax[e] + s]
        kz, ky, kx = np.nonzero(sub == 0)
        c = np.stack([kx + ax[e], ky + ay[e], kz + az[e]], axis=0).astype(np.float64)
        xs.append(lo[:, None] + (c + 0.5) * hmin)
        ls.append(np.full(c.shape, 0.5 * hmin))
    x = np.concatenate(xs, axis=1)
    l = np.concatenate(ls, axis=1)
    keep = np.ones(x.shape[1], dtype=bool)
    if w.keep is not None:
        keep &= w.keep(x[0], x[1], x[2])
    if w.drop_inside_body:
        keep &= ~_inside_body(w, x[0], x[1], x[2])
    x, l = x[:, keep], l[:, keep]
    if shuffle_seed is not None:
        p = np.random.default_rng(shuffle_seed).permutation(x.shape[1])
        x, l = x[:, p], l[:, p]
    return PointSet(np.ascontiguousarray(x), np.ascontiguousarray(l))


def jitter_points(w: Workload, ps: PointSet, k: int = 0) -> PointSet:
    """Move every centre by U[-l/2, l/2] per axis (seed 100+k), clipped so that the GIMP
    domain stays inside the mesh box. Exercises domains spanning several leaves."""
    rng = np.random.default_rng(100 + k)
    lo = np.asarray(w.lo, dtype=np.float64)[:, None]
    hi = lo + np.asarray(w.base, dtype=np.float64)[:, None] * w.h0
    d = rng.uniform(-0.5, 0.5, size=ps.x.shape) * ps.l
    x = np.clip(ps.x + d, lo + ps.l, hi - ps.l)
    return PointSet(np.ascontiguousarray(x), ps.l.copy())


def _det9(F):
    """Determinant of each 3x3 matrix stored row-major down the 9 rows of F (cofactor rule)."""
    return (F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6])
            + F[2] * (F[3] * F[7] - F[4] * F[6]))


def make_state(w: Workload, ps: PointSet, rho: float = 1.0) -> dict:
    """Material state per point (SoA float64). F_n = I + N(0, s^2) per entry, redrawn until
    det F_n > 0; b_n = F_n F_n^T stored as (xx, yy, zz, xy, yz, xz); J_n = det F_n."""
    n = ps.n
    rng = np.random.default_rng(w.seed_state)
    F = np.tile(np.eye(3).reshape(9, 1), (1, n))
    if w.Fn_std > 0:
        F = F + rng.normal(0.0, w.Fn_std, size=(9, n))
        while True:
            bad = np.nonzero(_det9(F) <= 0.0)[0]
            if bad.size == 0:
                break
            F[:, bad] = np.eye(3).reshape(9, 1) + rng.normal(0.0, w.Fn_std, size=(9, bad.size))
    # b_n = F F^T, rows of F are F[3r:3r+3]
    dot = lambda r, c: F[3 * r] * F[3 * c] + F[3 * r + 1] * F[3 * c + 1] + F[3 * r + 2] * F[3 * c + 2]
    bn = np.stack([dot(0, 0), dot(1, 1), dot(2, 2), dot(0, 1), dot(1, 2), dot(0, 2)], axis=0)
    Jn = _det9(F)
    vol = 8.0 * ps.l[0] * ps.l[1] * ps.l[2]
    full = lambda v: np.full(n, float(v))
    return dict(x=ps.x, l=ps.l, vol=vol, mass=rho * vol, Fn=np.ascontiguousarray(F),
                Jn=np.ascontiguousarray(Jn), bn=np.ascontiguousarray(bn),
                E=full(w.E), nu=full(w.nu), sy=full(w.sy))


def dirichlet_dofs(node_ijk: np.ndarray) -> np.ndarray:
    """uint8 mask over 3*n_node DOFs: nodes on the base z = lo_z are fixed in x, y and z."""
    node_ijk = np.asarray(node_ijk).reshape(-1, 3)
    fixed = node_ijk[:, 2] == 0
    return np.repeat(fixed, 3).astype(np.uint8)


def make_u(w: Workload, node_ijk: np.ndarray, k: int = 0, amp: float = 1e-3) -> np.ndarray:
    rng = np.random.default_rng([w.seed_u, 1, k])
    n = np.asarray(node_ijk).reshape(-1, 3).shape[0]
    u = rng.uniform(-amp, amp, size=3 * n)
    u[dirichlet_dofs(node_ijk).astype(bool)] = 0.0
    return u


def make_lambda(w: Workload, node_ijk: np.ndarray) -> np.ndarray:
    rng = np.random.default_rng([w.seed_lambda, 2])
    n = np.asarray(node_ijk).reshape(-1, 3).shape[0]
    lam = rng.normal(0.0, 1.0, size=3 * n)
    lam[dirichlet_dofs(node_ijk).astype(bool)] = 0.0
    return lam


def make_velocity(w: Workload, ps: PointSet, std: float = 0.1, seed: int = 6) -> np.ndarray:
    """Point velocities at the start of a step, [3][n], N(0, std^2) per component (seeded)."""
    rng = np.random.default_rng([seed, w.seed_state])
    return rng.normal(0.0, std, size=(3, ps.n))
