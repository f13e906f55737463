"""Shared setup of GPU parity tests: the same seeded inputs for the oracle and the library."""
from __future__ import annotations

import sys

import numpy as np
import torch

import workloads as W
from oracle.oracle import OracleMesh


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def build_pair(w, jitter=None, oracle_points=True):
    """Oracle mesh + points (from the oracle's leaves) and the library mesh on the same points."""
    from paper_2606_09275_amd.mesh import Mesh
    o = OracleMesh(w.crit())
    lv = o.leaves()
    ps = W.make_points(w, lv[:, :3], lv[:, 3])
    if jitter is not None:
        ps = W.jitter_points(w, ps, jitter)
    if oracle_points:
        o.set_points(ps.x, ps.l)
    log(f"[setup] {w.name} jitter={jitter} points={ps.n}")
    m = Mesh(w.crit(), torch.from_numpy(ps.x).cuda(), torch.from_numpy(ps.l).cuda())
    return o, m, ps


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max(initial=0.0))


def to_np(t):
    return t.detach().cpu().numpy()
