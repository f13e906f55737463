"""GPU check of the state permutation through the C ABI: dst[c][p] = src[c][perm[p]] bit for
bit, for component counts on both sides of the staged range (1, 2, 3, 6, 9, 18, 32, 33), with
a random permutation (staged record-major path), the mesh's own near-identity order and
permutations just below and just above the run-break threshold (direct path and staged
path)."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_common import log, to_np
from tests.helpers import tiny_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mesh():
    from paper_2606_09275_amd.mesh import Mesh
    w = tiny_workload("sphere", ppa=lambda lv: 12 if lv == 2 else 2)
    m0 = Mesh(w.crit())
    lv = to_np(m0.arrays()["leaf"])
    ps = W.jitter_points(w, W.make_points(w, lv[:, :3], lv[:, 3]), 1)
    m = Mesh(w.crit(), torch.from_numpy(ps.x).cuda(), torch.from_numpy(ps.l).cuda())
    log(f"[setup] permute mesh: {ps.n} points")
    return m


def _perms(n, rng):
    """Swapping two neighbours of the identity at a spot far from the others adds 3 run
    breaks: k // 3 swaps stay at or below the threshold n // 64, one more goes above it."""
    ident = np.arange(n)
    k = n // 64
    out = {"identity": ident, "random": rng.permutation(n)}
    spots = rng.choice(np.arange(4, n - 4, 8), size=k // 3 + 1, replace=False)
    for name, cnt in (("below", k // 3), ("above", k // 3 + 1)):
        p = ident.copy()
        for sp in spots[:cnt]:
            p[sp], p[sp + 1] = p[sp + 1], p[sp]
        out[name] = p
    return out


@pytest.mark.parametrize("ncomp", [1, 2, 3, 6, 9, 18, 32, 33])
def test_permute_bitexact(mesh, ncomp):
    n = mesh.info["n_point"]
    rng = np.random.default_rng(ncomp)
    src = rng.normal(size=(ncomp, n))
    sd = torch.from_numpy(src).cuda()
    own = to_np(mesh.arrays()["perm"])
    perms = _perms(n, rng)
    perms["mesh"] = own
    for name, p in perms.items():
        out = mesh.permute(sd, torch.from_numpy(p.astype(np.int64)).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(to_np(out).reshape(ncomp, n), src[:, p]), name
    log(f"[parity] permute ncomp={ncomp}: breaks below/above threshold "
        f"{int(np.sum(perms['below'][1:] != perms['below'][:-1] + 1))}/"
        f"{int(np.sum(perms['above'][1:] != perms['above'][:-1] + 1))} of n/64={n // 64}")
