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
        # The library reads every per-point field as float64. Parameters created as leaves
        # with requires_grad default to float32, so they are converted here; the shapes are
        # checked by Mesh.assemble before anything is launched.
        def f64(t):
            return t.detach().to(torch.float64).contiguous()

        s = dict(state)
        s.update(E=f64(E), nu=f64(nu), sy=f64(sy), vol=f64(vol))
        u64 = f64(u)
        out = mesh.assemble(s, u64, precision=precision, want_K=False, want_sigma=False, want_residual=False)
        ctx.mesh, ctx.state, ctx.u, ctx.precision = mesh, s, u64, precision
        ctx.dtypes = (E.dtype, nu.dtype, sy.dtype, vol.dtype)
        return out["f_int"]

    @staticmethod
    def backward(ctx, grad_f):
        g = ctx.mesh.adjoint(ctx.state, ctx.u, grad_f.detach().contiguous().to(torch.float64),
                             precision=ctx.precision)
        dt = ctx.dtypes
        return (None, None, None, g["dE"].to(dt[0]), g["dnu"].to(dt[1]), g["dsy"].to(dt[2]), g["dV"].to(dt[3]),
                None)
