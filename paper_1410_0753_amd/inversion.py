"""Differentiable gauge records for source inversion.

``GaugeRecords.apply(eta0, solver, nsteps, ckpt_every, u0, v0)`` runs the
split step from the initial surface eta0 (a free-surface deformation) and
velocities u0, v0 (optional; None = at rest) and returns the gauge records
[nrec][ng][3] (eta, u, v) as a tensor.  Its backward pass is the
library's adjoint (clf_adjoint_backward): frozen wet/dry decisions, a
checkpoint every ckpt_every steps (0: ceil(sqrt(nsteps))).  The map from
source coefficients to eta0 is ordinary torch (a linear combination of unit
sources), so autograd chains it with the adjoint.
"""
from __future__ import annotations

import torch


class GaugeRecords(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eta0, solver, nsteps, ckpt_every=0, u0=None, v0=None):
        solver.set_initial(eta0.detach(), None if u0 is None else u0.detach(),
                           None if v0 is None else v0.detach())
        solver.adjoint_forward(int(nsteps), int(ckpt_every))
        rec, _ = solver.read_gauges()
        ctx.solver = solver
        # the solver keeps the checkpoints of its last forward run only
        ctx.generation = solver.adjoint_generation
        ctx.has_uv = (u0 is not None, v0 is not None)
        return torch.from_numpy(rec).to(device=eta0.device, dtype=eta0.dtype)

    @staticmethod
    def backward(ctx, grad_rec):
        if ctx.solver.adjoint_generation != ctx.generation:
            raise RuntimeError("the solver ran another forward pass (GaugeRecords.apply or "
                               "adjoint_forward) after this one; its checkpoints are gone, so "
                               "this backward would use the later run's: give each pending "
                               "backward its own solver")
        d_eta0, d_u0, d_v0 = ctx.solver.adjoint_backward(
            grad_rec.detach().double().cpu().numpy())
        return (d_eta0, None, None, None, d_u0 if ctx.has_uv[0] else None,
                d_v0 if ctx.has_uv[1] else None)


def unit_sources_to_eta(coeffs, basis):
    """eta0 = sum_k c_k G_k (basis [K, ny, nx])."""
    return torch.tensordot(coeffs, basis, dims=1)
