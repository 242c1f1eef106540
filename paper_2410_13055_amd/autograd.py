"""torch.autograd bridge for the planner objective.

``CapacityCost.apply(eta, plan, scen, omega)`` returns the weighted mean
planner objective (1/|scen|) sum_s w_s h_s(x*_s(eta)) of the listed
scenarios (Section 2.1, eq. (1) without the investment term).  Forward runs
the library's batched dispatch solve; backward runs its capacity gradient
(Section 2.2: envelope pass plus, for an emissions weight, the adjoint
solve).  Torch only carries the K-vector between host and device.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gridplan


class CapacityCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eta: torch.Tensor, plan: "gridplan.Plan", scen, omega: float = 0.0,
                warm: int = 0):
        e = eta.detach().to("cpu", torch.float64).numpy().copy()
        cost, st, _ = plan.solve(e, scen, warm)
        w = np.array([plan.case.scenarios[s].weight for s in scen])
        emis = np.array([d["emis"] for d in st])
        h = float(np.mean(w * (cost + omega * emis)))
        ctx.plan, ctx.scen, ctx.omega, ctx.eta = plan, list(scen), float(omega), e
        return torch.tensor(h, dtype=eta.dtype, device=eta.device)

    @staticmethod
    def backward(ctx, gout: torch.Tensor):
        plan = ctx.plan
        try:
            g, _, _ = plan.grad(ctx.scen, ctx.omega)
        except gridplan.GridplanError as e:
            if e.code != gridplan.GP_ESTATE:
                raise
            # the plan solved another batch since forward: re-solve this one
            # from its stored solutions, then differentiate
            plan.solve(ctx.eta, ctx.scen, 1)
            g, _, _ = plan.grad(ctx.scen, ctx.omega)
        gt = torch.from_numpy(np.ascontiguousarray(g)).to(gout.device, gout.dtype)
        return gout * gt, None, None, None, None


def planning_objective(eta: torch.Tensor, plan, scen, gamma: torch.Tensor, omega: float = 0.0,
                       warm: int = 0) -> torch.Tensor:
    """gamma'eta + (1/|scen|) sum_s w_s h_s(x*_s(eta)) as a differentiable
    torch scalar (eq. (1))."""
    return (gamma * eta).sum() + CapacityCost.apply(eta, plan, scen, omega, warm)
