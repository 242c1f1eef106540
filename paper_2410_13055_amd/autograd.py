"""torch.autograd bridge for the planner objective.

``CapacityCost.apply(eta, plan, scen, omega)`` returns the weighted mean
planner objective (1/|scen|) sum_s w_s h_s(x*_s(eta)) of the listed
scenarios (Section 2.1, eq. (1) without the investment term).  Forward runs
the library's batched dispatch solve; backward runs its capacity gradient
(Section 2.2: envelope pass plus, for an emissions weight, the adjoint
solve).  Torch only carries the K-vector between host and device.
"""
from __future__ import annotations

import warnings

import numpy as np
import torch

from . import gridplan


class CapacityCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eta: torch.Tensor, plan: "gridplan.Plan", scen, omega: float = 0.0,
                warm: int = 0):
        e = eta.detach().to("cpu", torch.float64).numpy().copy()
        _, st, rc = plan.solve(e, scen, warm)
        if rc != gridplan.GP_OK:
            bad = [s for s, d in zip(scen, st) if d["status"]]
            warnings.warn(f"dispatch solves of scenarios {bad} missed the tolerance; the objective and its "
                          "gradient are those of the unconverged points", RuntimeWarning, stacklevel=2)
        h = plan.objective(scen, omega, eta=e)
        ctx.plan, ctx.scen, ctx.omega, ctx.eta = plan, list(scen), float(omega), e
        return torch.tensor(h, dtype=eta.dtype, device=eta.device)

    @staticmethod
    def backward(ctx, gout: torch.Tensor):
        plan = ctx.plan
        try:
            g, _, rc = plan.grad(ctx.scen, ctx.omega, eta=ctx.eta)
        except gridplan.GridplanError as e:
            if e.code != gridplan.GP_ESTATE:
                raise
            # the plan solved another batch or other capacities since
            # forward: re-solve this one from its stored solutions, then
            # differentiate
            plan.solve(ctx.eta, ctx.scen, 1)
            g, _, rc = plan.grad(ctx.scen, ctx.omega, eta=ctx.eta)
        if rc != gridplan.GP_OK:
            warnings.warn("the adjoint solve of the emissions gradient missed the tolerance; the gradient is "
                          "that of the unconverged adjoint point", RuntimeWarning, stacklevel=2)
        gt = torch.from_numpy(np.ascontiguousarray(g)).to(gout.device, gout.dtype)
        return gout * gt, None, None, None, None


def planning_objective(eta: torch.Tensor, plan, scen, gamma: torch.Tensor, omega: float = 0.0,
                       warm: int = 0) -> torch.Tensor:
    """gamma'eta + (1/|scen|) sum_s w_s h_s(x*_s(eta)) as a differentiable
    torch scalar (eq. (1))."""
    return (gamma * eta).sum() + CapacityCost.apply(eta, plan, scen, omega, warm)
