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

A planner objective on the prices, h = lmp * sum pi D (Section 2.1 allows
h_s to depend on the LMPs), needs the derivative of the dual solution: on
the same system dy = -r (E_F E_F')^+ E_A dx_A, so with
    v = (E_F E_F')^+ g_y,   g_y = lmp * D on the balance rows,
    dl/dx_A = -r E_A' v,
chained through the active bounds like the primal part.

When the constraint matrix depends on the capacities (Section 2.1's
A_s(eta); here a line's susceptance beta_l(eta_l) in its flow rows), the
perturbed system gains the terms of dE: with G = dE'y,
    r dx_F - E_F' dy = G_F,   E_F dx_F + E_A dx_A = -dE x,
and the same adjoint w gives
    dl/d eta_j (extra) = -w' dE_j x + (1/r) (g - E'w)_F' (dE_j' y)_F,
which for h = c (w = y, zero residual) is the envelope term -y' dE_j x.

A capacity at zero collapses its boxes to points (a generator with
eta_g = 0, a line with eta_l = 0).  The map is then one-sided in eta, and
the derivative returned is the one for increasing capacity: an entry whose
multiplier z_i is positive would move to the bound that opens, so it counts
as held at that bound (the upper one; for a line with z_i < 0 the lower one,
-eta_l), and an entry with z_i <= 0 stays where it is.

The map x*(eta) is piecewise affine, so the planner objective is piecewise
quadratic: on every segment of capacities over which the active set stays
optimal it is a quadratic, and a central difference along such a segment is
its exact derivative.  ``fixed_set_differences`` evaluates that difference
by re-solving the equality system of the active set at eta_j +- h (one
factorisation, two back-solves per capacity) and verifying the optimality
signs at both ends; a coordinate whose verification fails on either side
has a kink within h of eta: the map is not differentiable there (Section
2.2 assumes differentiability).
"""
from __future__ import annotations

import numpy as np

from . import dispatch as D


def loss_gradient_x(qp: D.QP, x: np.ndarray, omega: float) -> np.ndarray:
    """grad h(x) = r x + q + omega * emissions-rate."""
    return qp.r * x + qp.q + omega * qp.emis


def _dependent(qp: D.QP):
    """Entries whose upper / lower bound is a nonzero multiple of a capacity."""
    dep_hi = (qp.hi_idx >= 0) & (qp.hi_coef != 0)
    dep_lo = (qp.lo_idx >= 0) & (qp.lo_coef != 0)
    return dep_hi, dep_lo


def _collapsed(qp: D.QP):
    """Entries whose box is a single point."""
    return np.isfinite(qp.lo) & np.isfinite(qp.hi) & (qp.hi - qp.lo <= 1e-12 * (1 + np.abs(qp.hi)))


def capacity_sides(qp: D.QP, sol: D.Solution):
    """Active sets used for the derivative (see the module docstring): the
    solution's own classification, except at boxes collapsed by a zero
    capacity, where the sign of the multiplier picks the side that opens
    (a generator with z_i <= 0 stays at its fixed lower bound 0 and
    contributes nothing)."""
    at_lo = sol.active_lo.copy()
    at_hi = sol.active_hi.copy()
    dep_hi, dep_lo = _dependent(qp)
    coll = _collapsed(qp) & (dep_hi | dep_lo)
    up = coll & dep_hi & (sol.z > 0)
    at_hi[coll] = up[coll]
    at_lo[coll] = ~up[coll]
    return at_lo, at_hi


def eta_from_active(qp: D.QP, dl_dx: np.ndarray, at_lo: np.ndarray, at_hi: np.ndarray) -> np.ndarray:
    """Chain rule through the active bounds: sum_i a_i dl/dx_i per capacity."""
    out = np.zeros(qp.K)
    m = at_hi & (qp.hi_idx >= 0)
    np.add.at(out, qp.hi_idx[m], qp.hi_coef[m] * dl_dx[m])
    m = at_lo & (qp.lo_idx >= 0) & ~at_hi
    np.add.at(out, qp.lo_idx[m], qp.lo_coef[m] * dl_dx[m])
    return out


def matrix_terms(qp: D.QP, x: np.ndarray, y: np.ndarray, w: np.ndarray, res: np.ndarray) -> np.ndarray:
    """The capacity derivative's terms from dE (module docstring): for an
    AC line l with d beta_l / d eta_l = b', its flow rows (l, t) hold
    -beta_l at th[from] and +beta_l at th[to], so
        -w' dE_l x = b' sum_t w_(l,t) (th_from - th_to),
        (1/r) res' dE_l' y = -(b' / r) sum_t y_(l,t) (res_th_from - res_th_to)
    with res = g - E'w (angles are always free)."""
    d = qp.dims
    T, Lac, G = d["T"], d["Lac"], d["G"]
    vs, rs = d["vs"], d["rs"]
    out = np.zeros(qp.K)
    if Lac == 0:
        return out
    th = x[vs["th"]].reshape(-1, T)
    rth = res[vs["th"]].reshape(-1, T)
    lf, lt = d["line_from"][:Lac], d["line_to"][:Lac]
    wl = w[rs["flow"]].reshape(Lac, T)
    yl = y[rs["flow"]].reshape(Lac, T)
    db = qp.line_dbeta[:Lac]
    out[G:G + Lac] = db * ((wl * (th[lf] - th[lt])).sum(1) - (yl * (rth[lf] - rth[lt])).sum(1) / qp.r)
    return out


def lmp_dl_dx(qp: D.QP, free: np.ndarray, lmp: float) -> np.ndarray:
    """-r E' v with (E_F E_F') v = lmp * D (balance rows): the derivative of
    lmp * pi'D with respect to the held entries (module docstring)."""
    _, _, msolve, _ = D._free_factor(qp, free)
    gy = np.zeros(qp.m)
    rs = qp.dims["rs"]["bal"]
    gy[rs] = lmp * qp.e[rs]
    return -qp.r * (qp.E.T @ msolve(gy))


def scenario_gradient(qp: D.QP, sol: D.Solution, omega: float, lmp: float = 0.0) -> dict:
    """d h_s(x*(eta)) / d eta for one scenario via the least-squares adjoint.

    Returns the gradient, the envelope value (cost part only), the adjoint w
    and a flag for points where the map is not differentiable (weakly active
    bounds, or a solution whose active set the polish could not settle; there
    the value is one element of the generalised gradient)."""
    at_lo, at_hi = capacity_sides(qp, sol)
    free = ~(sol.active_lo | sol.active_hi)
    g = loss_gradient_x(qp, sol.x, omega)
    w, rankdef = D.adjoint_lsq(qp, free, g)
    dl_dx = g - qp.E.T @ w
    grad = eta_from_active(qp, dl_dx, at_lo, at_hi)
    env = eta_from_active(qp, -sol.z, at_lo, at_hi)
    if qp.line_dbeta is not None:
        grad += matrix_terms(qp, sol.x, sol.y, w, dl_dx)
        env += matrix_terms(qp, sol.x, sol.y, sol.y, np.zeros(qp.n))
    if lmp:
        if qp.line_dbeta is not None:
            raise NotImplementedError("price objectives with a capacity-dependent matrix")
        grad += eta_from_active(qp, lmp_dl_dx(qp, free, lmp), at_lo, at_hi)
    # weakly active entries whose bound depends on a capacity make the map kinked
    bscale = 1.0 + np.abs(qp.q).max()
    dep_hi, dep_lo = _dependent(qp)
    dep = (sol.active_hi & dep_hi) | (sol.active_lo & dep_lo)
    weak = dep & ~_collapsed(qp) & (np.abs(sol.z) < 1e-7 * bscale)
    return dict(grad=grad, envelope=env, w=w, dl_dx=dl_dx, kink=bool(weak.any() or not sol.polished),
                rank_deficient=rankdef)


def fixed_set_differences(qp: D.QP, sol: D.Solution, omega: float, h: float = 1e-3, js=None,
                          tol_x: float = 1e-9, tol_z: float = 1e-9, lmp: float = 0.0) -> dict:
    """Central differences of h_s along each capacity j in ``js`` (default
    all), from re-solves with the solution's active set held fixed.

    At eta +- h e_j the active entries sit at their moved bounds and the free
    entries solve  r x_F + q_F = E_F' y,  E_F x_F = e - E_A x_A  (the reduced
    system does not depend on eta, only its right-hand side does, so one
    factorisation serves every coordinate).  Each end is accepted only if it
    is optimal: free entries inside their moved box and every held entry's
    multiplier with the right sign.  Returns per coordinate the central,
    forward and backward differences and ``ok`` (both ends verified; then the
    central difference is the exact derivative of the quadratic piece), the
    distance to the nearest kink along the coordinate (``dist``: the largest
    step, either way, for which the active set stays optimal, from a ratio
    test on the step direction) and the curvature of h along it
    (``curv`` = d2h/deta_j2 on the piece)."""
    if not sol.polished:
        raise ValueError("fixed-active-set differences need a polished solution")
    if qp.line_dbeta is not None:
        raise NotImplementedError("the reduced system moves with eta when the constraint matrix does")
    K = qp.K
    js = np.arange(K) if js is None else np.asarray(js)
    at_lo, at_hi = sol.active_lo, sol.active_hi
    free = ~(at_lo | at_hi)
    E = qp.E.tocsc()
    EF, EA, msolve, _ = D._free_factor(qp, free)
    EAc = E[:, ~free]
    x0, z0 = sol.x, sol.z
    g0 = loss_gradient_x(qp, x0, omega)
    bscale = 1.0 + np.abs(qp.q).max()
    xs = 1.0 + max(np.abs(qp.lo[np.isfinite(qp.lo)]).max(initial=0.0),
                   np.abs(qp.hi[np.isfinite(qp.hi)]).max(initial=0.0))
    coll = _collapsed(qp)
    idx_free = np.where(free)[0]
    out = dict(central=np.zeros(len(js)), forward=np.zeros(len(js)), backward=np.zeros(len(js)),
               ok=np.zeros(len(js), bool), ok_plus=np.zeros(len(js), bool), ok_minus=np.zeros(len(js), bool),
               dist=np.zeros(len(js)), curv=np.zeros(len(js)))
    held_hi = ~free & ~coll & at_hi
    held_lo = ~free & ~coll & at_lo & ~at_hi
    fin_lo, fin_hi = np.isfinite(qp.lo), np.isfinite(qp.hi)
    rs_bal = qp.dims["rs"]["bal"]

    def ratio(num, den):
        """min over den > 0 of num / den (inf when none)."""
        m = den > 0
        return float(np.min(np.maximum(num[m], 0.0) / den[m])) if m.any() else np.inf
    for k, j in enumerate(js):
        # bound movement per unit capacity (a_i where the bound is a_i eta_j)
        dhi = np.where(qp.hi_idx == j, qp.hi_coef, 0.0)
        dlo = np.where(qp.lo_idx == j, qp.lo_coef, 0.0)
        dxA = np.where(at_hi, dhi, np.where(at_lo, dlo, 0.0))
        # r dx_F = E_F' dy,  E_F dx_F = -E_A dx_A
        dy = -qp.r * msolve(EAc @ dxA[~free])
        dx = dxA.copy()
        dx[free] = (EF.T @ dy) / qp.r
        dz = E.T @ dy - qp.r * dx
        oks = []
        for sgn in (1.0, -1.0):
            x = x0 + sgn * h * dx
            z = z0 + sgn * h * dz
            lo = qp.lo + sgn * h * dlo
            hi = qp.hi + sgn * h * dhi
            inside = np.all((x[idx_free] >= lo[idx_free] - tol_x * xs) & (x[idx_free] <= hi[idx_free] + tol_x * xs))
            held = ~free & ~coll
            signs = np.all(z[held & at_hi] >= -tol_z * bscale) and np.all(z[held & at_lo & ~at_hi] <= tol_z * bscale)
            oks.append(bool(inside and signs))
        # distance to the nearest kink: free entries meeting a (moving)
        # bound, held entries whose multiplier reaches zero
        dists = []
        for sgn in (1.0, -1.0):
            f = free
            d_hi = ratio((qp.hi - x0)[f & fin_hi], (sgn * (dx - dhi))[f & fin_hi])
            d_lo = ratio((x0 - qp.lo)[f & fin_lo], (sgn * (dlo - dx))[f & fin_lo])
            d_zh = ratio(z0[held_hi], (-sgn * dz)[held_hi])
            d_zl = ratio(-z0[held_lo], (sgn * dz)[held_lo])
            dists.append(min(d_hi, d_lo, d_zh, d_zl))
        out["dist"][k] = min(dists)
        out["curv"][k] = qp.r * float(dx @ dx)
        # h(x0 + s h dx) - h(x0) = s h g0'dx + (r/2) h^2 ||dx||^2  (exact for the quadratic)
        lin = float(g0 @ dx) + (lmp * float(qp.e[rs_bal] @ dy[rs_bal]) if lmp else 0.0)
        quad = 0.5 * qp.r * h * h * float(dx @ dx)
        vp, vm = h * lin + quad, -h * lin + quad
        out["central"][k] = (vp - vm) / (2 * h)
        out["forward"][k] = vp / h
        out["backward"][k] = -vm / h
        out["ok_plus"][k], out["ok_minus"][k] = oks
        out["ok"][k] = oks[0] and oks[1]
    out["js"] = js
    return out


def batch_gradient(case, eta: np.ndarray, scen, omega: float, tol: float = 1e-10, lmp: float = 0.0):
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
        gr = scenario_gradient(qp, sol, omega, lmp)
        out[a:b] += sc.weight * gr["grad"]
        h = D.planner_objective(qp, sol.x, omega, sol.y, lmp)
        hbar += sc.weight * h
        per.append(dict(qp=qp, sol=sol, grad=gr, h=h))
    nb = len(scen)
    return out / nb, hbar / nb, per


def value(case, s: int, eta_net: np.ndarray, omega: float, tol: float = 1e-10, lmp: float = 0.0) -> float:
    """h_s(x*_s(eta)) from a full polished re-solve."""
    qp = D.assemble(case, s, eta_net)
    sol = D.solve(qp, tol=tol)
    return D.planner_objective(qp, sol.x, omega, sol.y, lmp)


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
