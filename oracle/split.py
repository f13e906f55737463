"""Oracle: splitting of refined GIMPs (Section 5, GIMP refinement and the transfer of their data).
TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.

A split GIMP becomes 8 GIMPs that tile its domain: child c (bits c_0, c_1, c_2 for the axes)
is centred at x_a + s_a l_a / 2 with s_a = -1 if bit a is clear and +1 if set, and has half
sides l / 2, volume V / 8 and mass m / 8. Data that is constant over the GIMP's domain
(deformation gradient, its determinant, elastic left Cauchy-Green tensor, velocity, material
parameters) is copied to the eight children. Data defined by the reference position is
evaluated at the child's own reference position: F is constant over the domain, so the
current-to-reference map is affine there and X_c = X + F_n^{-1} (x_c - x).

Material parameters given by the reference position are affine functions here,
theta(X) = a_0 + a_1 X_1 + a_2 X_2 + a_3 X_3 (the paper's example is E = 1 - z).

The output keeps the input order: an unsplit point, or a split point's 8 children in child
order.
"""
from __future__ import annotations

import numpy as np

PER_POINT = {"x": 3, "l": 3, "vol": 1, "mass": 1, "Jn": 1, "bn": 6, "Fn": 9, "E": 1, "nu": 1, "sy": 1}
PROPS = ("E", "nu", "sy")


def split_points(s: dict, split: np.ndarray, X: np.ndarray | None = None, v: np.ndarray | None = None,
                 props: dict | None = None) -> dict:
    """s: per-point arrays ([c][n] or [n]) of PER_POINT; split: [n] flags; X, v: [3][n] reference
    positions and velocities (optional); props: {name: (a0, a1, a2, a3)} for the material
    parameters defined by the reference position (needs X and F_n). Returns the new arrays
    (with "X" and "v" when given)."""
    split = np.asarray(split).astype(bool)
    n = split.shape[0]
    props = props or {}
    if props and (X is None or "Fn" not in s):
        raise ValueError("material parameters given by the reference position need X and F_n")
    out = {k: [] for k in PER_POINT if k in s}
    if X is not None:
        out["X"] = []
    if v is not None:
        out["v"] = []
    for p in range(n):
        rec = {k: np.asarray(s[k], np.float64).reshape(PER_POINT[k], n)[:, p].copy() for k in out if k in PER_POINT}
        if X is not None:
            rec["X"] = np.asarray(X, np.float64)[:, p].copy()
        if v is not None:
            rec["v"] = np.asarray(v, np.float64)[:, p].copy()
        if not split[p]:
            for k in out:
                out[k].append(rec[k])
            continue
        Finv = np.linalg.inv(rec["Fn"].reshape(3, 3)) if X is not None and "Fn" in rec else None
        for c in range(8):
            ch = {k: val.copy() for k, val in rec.items()}
            sgn = np.array([1.0 if (c >> a) & 1 else -1.0 for a in range(3)])
            ch["x"] = rec["x"] + sgn * (rec["l"] / 2.0)
            ch["l"] = rec["l"] / 2.0
            ch["vol"] = rec["vol"] / 8.0
            ch["mass"] = rec["mass"] / 8.0
            if X is not None:
                ch["X"] = rec["X"] + Finv @ (ch["x"] - rec["x"])
                for name, a in props.items():
                    ch[name] = np.array([a[0] + a[1] * ch["X"][0] + a[2] * ch["X"][1] + a[3] * ch["X"][2]])
            for k in out:
                out[k].append(ch[k])
    res = {}
    for k, rows in out.items():
        arr = np.array(rows, np.float64).reshape(len(rows), -1).T
        res[k] = arr.reshape(-1) if arr.shape[0] == 1 else np.ascontiguousarray(arr)
    return res
