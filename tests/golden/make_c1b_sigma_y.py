"""Writes c1b_sigma_y.json: the yield stress of the partial-yielding sphere workload.

Rule: the yield stress is the 70th percentile of the trial von Mises stress sqrt(3 J2) of the
FP64 oracle over the sphere workload's points (mesh, points, state and displacement of the
sphere workload, which has the same inputs apart from the yield stress), so that 30 % of the
points yield (Section 2.2: perfect plasticity, von Mises surface). Only the oracle is called.

Run from the repository root:  python tests/golden/make_c1b_sigma_y.py
"""
from __future__ import annotations

import json
import math
import sys
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import workloads as W  # noqa: E402
from oracle.oracle import OracleMesh  # noqa: E402

OUT = Path(__file__).resolve().parent / "c1b_sigma_y.json"


def trial_q(w):
    o = OracleMesh(w.crit())
    lv = o.leaves()
    ps = W.make_points(w, lv[:, :3], lv[:, 3])
    o.set_points(ps.x, ps.l)
    st = W.make_state(w, ps)
    st["sy"] = np.full(ps.n, math.inf)
    u = W.make_u(w, o.nodes())
    return o.assemble(st, u, want_K=False)["q_trial"]


def main():
    w = W.get("c1")
    q = trial_q(w)
    sy = float(np.percentile(q, 70))
    rec = dict(workload="sphere workload (C1 mesh, points, state, displacement)", n_point=int(q.size),
               rule="70th percentile of the oracle's trial von Mises stress", sigma_y=sy,
               yield_fraction=float(np.mean(q > sy)), q_trial_median=float(np.median(q)))
    OUT.write_text(json.dumps(rec, indent=2) + "\n")
    print(json.dumps(rec, indent=2))


if __name__ == "__main__":
    main()
