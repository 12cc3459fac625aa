"""Differentiable solve: flux and pressure as functions of the per-cell log-permeability.

Forward: nu = exp(-log K) -> vem_set_coefficient -> vem_solve.  Backward
(adjoint method): solve K lambda = [dJ/du; dJ/dp] with the same operator and
preconditioner (K is symmetric), then dJ/d(log K_P) = nu_P lambda_P^T M1_P u_P
from vem_coefficient_gradient.  Every numerical step runs in the HIP library.
"""

from __future__ import annotations

import torch


class FluxPressureFromLogK(torch.autograd.Function):
    @staticmethod
    def forward(ctx, logk, solver, solve_kw):
        if solver.boundary != "pressure":
            raise ValueError("the adjoint gradient supports pressure boundary data only")
        solver.set_coefficient(torch.exp(-logk.detach()))
        u, p, info = solver.solve(**solve_kw)
        if not info["converged"]:
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.solver, ctx.solve_kw = solver, solve_kw
        ctx.save_for_backward(logk.detach(), u)
        return u, p

    @staticmethod
    def backward(ctx, grad_u, grad_p):
        logk, u = ctx.saved_tensors
        s = ctx.solver
        sz = s.sizes()
        if grad_u is None:
            grad_u = torch.zeros(sz["n_u"], dtype=torch.float64, device=u.device)
        if grad_p is None:
            grad_p = torch.zeros(sz["n_p"], dtype=torch.float64, device=u.device)
        # the solver may have been given another coefficient since the forward pass
        s.set_coefficient(torch.exp(-logk))
        rhs = torch.cat([grad_u.to(torch.float64).contiguous(), grad_p.to(torch.float64).contiguous()])
        lu, lp, info = s.solve(rhs=rhs, **ctx.solve_kw)
        if not info["converged"]:
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        return s.coefficient_gradient(u, lu), None, None


def solve_logk(solver, logk, **solve_kw):
    """(u, p) = solve with nu = exp(-logk); differentiable with respect to logk."""
    return FluxPressureFromLogK.apply(logk, solver, solve_kw)
