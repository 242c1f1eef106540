"""Implicit gradient of the planner objective with respect to capacities.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.2 of the paper writes the planning gradient as
    Delta = gamma + (1/S) sum_s (d x*_s / d eta)' grad h_s(x*_s),
and obtains the Jacobian of the argmin from the implicit function theorem on
the dispatch problem's optimality conditions.  Only the vector-Jacobian
product is ever needed.  On the active-set KKT system of the QP in
``dispatch`` (Hessian r I, box bounds some of which equal a_i * eta_j):

    free set F, active set A (entries held at a bound),
    r dx_F - E_F' dy = 0,  E_F dx_F + E_A dx_A = 0,  dx_A = a_A d eta,

which gives, for a loss l with gradient g = grad h(x*),
    w = argmin_w || E_F' w - g_F ||            (least-squares adjoint)
    dl/dx_A = g_A - E_A' w
    dl/d eta_j = sum over active i whose bound is a_i eta_j of a_i dl/dx_i.

For h = c (no emissions weight) the fit is exact with w = y*, so
dl/dx_A = -z_A and the gradient is the envelope-theorem value
-sum_i a_i z_i (z the box multipliers); that identity is a pin.
"""
from __future__ import annotations

import numpy as np

from . import dispatch as D


def loss_gradient_x(qp: D.QP, x: np.ndarray, omega: float) -> np.ndarray:
    """grad h(x) = r x + q + omega * emissions-rate."""
    return qp.r * x + qp.q + omega * qp.emis


def eta_from_active(qp: D.QP, dl_dx: np.ndarray, at_lo: np.ndarray, at_hi: np.ndarray) -> np.ndarray:
    """Chain rule through the active bounds: sum_i a_i dl/dx_i per capacity."""
    out = np.zeros(qp.K)
    m = at_hi & (qp.hi_idx >= 0)
    np.add.at(out, qp.hi_idx[m], qp.hi_coef[m] * dl_dx[m])
    m = at_lo & (qp.lo_idx >= 0) & ~at_hi
    np.add.at(out, qp.lo_idx[m], qp.lo_coef[m] * dl_dx[m])
    return out


def scenario_gradient(qp: D.QP, sol: D.Solution, omega: float) -> dict:
    """d h_s(x*(eta)) / d eta for one scenario via the least-squares adjoint.

    Returns the gradient, the envelope value (cost part only), the adjoint w
    and a flag for points where the map is not differentiable (weakly active
    bounds, or a solution whose active set the polish could not settle; there
    the value is one element of the generalised gradient)."""
    at_lo, at_hi = sol.active_lo, sol.active_hi
    free = ~(at_lo | at_hi)
    g = loss_gradient_x(qp, sol.x, omega)
    w, rankdef = D.adjoint_lsq(qp, free, g)
    dl_dx = g - qp.E.T @ w
    grad = eta_from_active(qp, dl_dx, at_lo, at_hi)
    env = eta_from_active(qp, -sol.z, at_lo, at_hi)
    # weakly active entries whose bound depends on a capacity make the map kinked
    bscale = 1.0 + np.abs(qp.q).max()
    dep = ((at_hi & (qp.hi_idx >= 0) & (qp.hi_coef != 0)) |
           (at_lo & (qp.lo_idx >= 0) & (qp.lo_coef != 0)))
    fixed = np.isfinite(qp.lo) & np.isfinite(qp.hi) & (qp.hi - qp.lo <= 1e-12 * (1 + np.abs(qp.hi)))
    weak = dep & ~fixed & (np.abs(sol.z) < 1e-7 * bscale)
    return dict(grad=grad, envelope=env, w=w, dl_dx=dl_dx, kink=bool(weak.any() or not sol.polished),
                rank_deficient=rankdef)


def batch_gradient(case, eta: np.ndarray, scen, omega: float, tol: float = 1e-10):
    """(1/|scen|) sum_s w_s d h_s / d eta over the listed scenarios, on the
    case-wide capacity vector (investment term gamma excluded).  Also returns
    the weighted mean planner objective and per-scenario results."""
    off = case.eta_offsets()
    out = np.zeros(case.K)
    hbar = 0.0
    per = []
    for s in scen:
        sc = case.scenarios[s]
        a, b = off[sc.network], off[sc.network + 1]
        qp = D.assemble(case, s, eta[a:b])
        sol = D.solve(qp, tol=tol)
        gr = scenario_gradient(qp, sol, omega)
        out[a:b] += sc.weight * gr["grad"]
        h = D.planner_objective(qp, sol.x, omega)
        hbar += sc.weight * h
        per.append(dict(qp=qp, sol=sol, grad=gr, h=h))
    nb = len(scen)
    return out / nb, hbar / nb, per


def value(case, s: int, eta_net: np.ndarray, omega: float, tol: float = 1e-10) -> float:
    """h_s(x*_s(eta)) from a full polished re-solve."""
    qp = D.assemble(case, s, eta_net)
    sol = D.solve(qp, tol=tol)
    return D.planner_objective(qp, sol.x, omega)


def central_difference(case, s: int, eta_net: np.ndarray, j: int, omega: float,
                       h: float = 1e-3, tol: float = 1e-10) -> dict:
    """Central, forward and backward differences of h_s along capacity j with
    full re-solves (a coordinate where forward and backward disagree is a
    kink)."""
    e0 = value(case, s, eta_net, omega, tol)
    ep = eta_net.copy()
    ep[j] += h
    em = eta_net.copy()
    em[j] -= h
    vp = value(case, s, ep, omega, tol)
    vm = value(case, s, em, omega, tol)
    return dict(central=(vp - vm) / (2 * h), forward=(vp - e0) / h, backward=(e0 - vm) / h)
