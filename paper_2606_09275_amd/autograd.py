"""torch.autograd.Function over the assembly: f_int(E, nu, sigma_y, V_n) with its hand-written
adjoint as the backward pass (parameter calibration)."""
from __future__ import annotations

import torch

from .mesh import Mesh


class MPMForce(torch.autograd.Function):
    """forward(mesh, state, u, E, nu, sy, vol, precision) -> f_int (FP64, [n_dof]).

    `state` holds the remaining sorted-order point arrays (x, l, mass, Jn, bn, g); E, nu,
    sy, vol are [n] device tensors. backward(dL/df_int) runs the adjoint assembly with
    lambda = dL/df_int and returns dL/dE, dL/dnu, dL/dsy, dL/dvol per point (the return map
    is recomputed, nothing is stored by the forward pass)."""

    @staticmethod
    def forward(ctx, mesh: Mesh, state: dict, u, E, nu, sy, vol, precision="f64"):
        s = dict(state)
        s.update(E=E.detach().contiguous(), nu=nu.detach().contiguous(), sy=sy.detach().contiguous(),
                 vol=vol.detach().contiguous())
        out = mesh.assemble(s, u.detach().contiguous(), precision=precision, want_K=False, want_sigma=False,
                            want_residual=False)
        ctx.mesh, ctx.state, ctx.u, ctx.precision = mesh, s, u.detach().contiguous(), precision
        return out["f_int"]

    @staticmethod
    def backward(ctx, grad_f):
        g = ctx.mesh.adjoint(ctx.state, ctx.u, grad_f.detach().contiguous().to(torch.float64),
                             precision=ctx.precision)
        return None, None, None, g["dE"], g["dnu"], g["dsy"], g["dV"], None
