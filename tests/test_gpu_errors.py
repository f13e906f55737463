"""Error paths of the C ABI, forced from the host with invalid inputs that the library's own
checks turn into status codes (every kernel still runs to completion)."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from paper_2606_09275_amd._lib import MPM_EARG, MPM_EDET, MPM_ENONFINITE, MPM_EOUTSIDE, MPMError
from tests.gpu_common import build_pair
from tests.helpers import tiny_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prob():
    w = tiny_workload("sphere", E=1e4, nu=0.3, sy=40.0, Fn_std=0.02)
    o, m, ps = build_pair(w, jitter=0, oracle_points=False)
    st = W.make_state(w, ps)
    nodes = m.arrays()["node_ijk"].cpu().numpy()
    return w, m, ps, m.sorted_state(st), nodes


def test_inverted_point_reports_det(prob):
    w, m, ps, s, nodes = prob
    u = torch.from_numpy(W.make_u(w, nodes, amp=5.0)).cuda()
    with pytest.raises(MPMError) as ei:
        m.assemble(s, u, "f64")
    assert ei.value.code == MPM_EDET and ei.value.index >= 0
    # the handle stays usable after an error
    m.assemble(s, torch.zeros_like(u), "f64")


def test_nonfinite_displacement(prob):
    w, m, ps, s, nodes = prob
    u = torch.from_numpy(W.make_u(w, nodes)).cuda()
    u[3 * 5] = float("nan")
    for prec in ("f64", "f32k"):
        with pytest.raises(MPMError) as ei:
            m.assemble(s, u, prec)
        assert ei.value.code in (MPM_ENONFINITE, MPM_EDET)
    with pytest.raises(MPMError):
        m.adjoint(s, u, torch.ones_like(u), "f64")


def test_bad_precision_and_sizes(prob):
    w, m, ps, s, nodes = prob
    u = torch.zeros(m.info["n_dof"], dtype=torch.float64, device="cuda")
    with pytest.raises(MPMError) as ei:
        m.assemble(s, u, 7)
    assert ei.value.code == MPM_EARG
    with pytest.raises(MPMError) as ei:
        m.point_sort(s["x"][:, :10].contiguous())
    assert ei.value.code == MPM_EARG


def test_point_outside_mesh():
    from paper_2606_09275_amd.mesh import Mesh
    w = tiny_workload("sphere")
    x = np.array([[0.5], [0.5], [0.99]])
    l = np.array([[0.05], [0.05], [0.05]])
    with pytest.raises(MPMError) as ei:
        Mesh(w.crit(), torch.from_numpy(x).cuda(), torch.from_numpy(l).cuda())
    assert ei.value.code == MPM_EOUTSIDE
