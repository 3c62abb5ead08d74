"""Differentiable utilisation: U(kappa, q) with a hand-written discrete adjoint backward.

The forward is the steady solve of the SOC transport equation at reaction activity kappa
(per voxel; lam = Da kappa n_f) and flow rate q (u = q u0, the Stokes-regime scaling of
one flow field), returning U of Eq. (utilization-def).  The steady state is the solution
of a linear system A s = b, so its gradient needs no time checkpointing: one adjoint solve
A^T psi = dU/ds (the same stencil with reversed advection, run by the library) gives
    dU/dkappa_P = Da n_f(P) psi_P (s_eq - s_P),     dU/dq = psi . Radv(s; u0).
"""
from __future__ import annotations

import torch

from . import socfv


class SocSteady(torch.autograd.Function):
    """U = SocSteady.apply(kappa, q, problem, params).

    kappa: CUDA float32 (nz, ny, nx) activity; q: float64 scalar tensor (flow-rate scale);
    problem: socfv.Problem (geometry + u0); params: socfv.Params (FINITE_RATE).
    """

    @staticmethod
    def forward(ctx, kappa, q, problem, params):
        problem.set_flow_rate(float(q))
        problem.set_activity(kappa.detach().contiguous())
        _, st = socfv.solve_soc_steady(problem.ctx, params, want_state=False)
        ctx.problem = problem
        ctx.params = params
        ctx.q = float(q)
        ctx.kappa = kappa.detach()
        ctx.stats = st
        return torch.tensor(st.U, dtype=torch.float64, device=kappa.device)

    @staticmethod
    def backward(ctx, gU):
        pb = ctx.problem
        # the context holds the state of its last solve; redo the forward if it moved on
        if pb.q != ctx.q or pb.kappa is None or pb.kappa.data_ptr() != ctx.kappa.data_ptr():
            pb.set_flow_rate(ctx.q)
            pb.set_activity(ctx.kappa.contiguous())
            socfv.solve_soc_steady(pb.ctx, ctx.params, want_state=False)
        g, dlnq, _, _ = socfv.solve_soc_adjoint(pb.ctx, ctx.params, want_grad=True)
        gk = (gU * g).to(ctx.kappa.dtype) if ctx.needs_input_grad[0] else None
        gq = None
        if ctx.needs_input_grad[1]:
            gq = (gU * (dlnq / ctx.q)).to(torch.float64)
        return gk, gq, None, None


def utilisation(kappa, q, problem, params):
    return SocSteady.apply(kappa, q, problem, params)
