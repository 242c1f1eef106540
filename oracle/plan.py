"""Planner objective, projected gradient step and the joint-QP pin.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.1, eq. (1): Phi(eta) = gamma'eta + (1/S) sum_s w_s h_s(x*_s(eta))
over eta_min <= eta <= eta_max.  Section 2.2: Delta = gamma + (1/S) sum_s
(dx*_s)' grad h_s and eta <- proj(eta - alpha Delta); with B sampled
scenarios the average runs over the sample.

When h_s = c_s (no emissions weight) the paper notes the bilevel problem is
the classical joint problem over (eta, x_1..x_S) (Section 2.1, the remark on
vertically integrated utilities); ``joint_optimum`` solves that convex QP
directly, which pins what planning with the implicit gradient must approach.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import dispatch as D
from . import gradient as Gm


def phi(case, eta, scen, omega):
    """Phi over the listed scenarios and its gradient Delta."""
    g, hbar, _ = Gm.batch_gradient(case, eta, scen, omega)
    gam = case.gamma()
    return float(gam @ eta + hbar), gam + g


def projected_step(case, eta, alpha, scen, omega):
    """One step of Section 2.2: returns (new eta, Phi(eta), Delta)."""
    f, d = phi(case, eta, scen, omega)
    return np.clip(eta - alpha * d, case.eta_min(), case.eta_max()), f, d


def joint_optimum(case, scen=None):
    """min gamma'eta + (1/|scen|) sum_s w_s c_s(x_s) over (eta, x_s) with every
    capacity-dependent bound written as a linear inequality through a slack:
    x_i + s_i = a_i eta_j (upper) or x_i - s_i = a_i eta_j (lower), s >= 0.
    Solved with the same interior-point method (diagonal Hessian with zeros on
    eta and the slacks, which are bounded).  Single-network cases only."""
    assert len(case.networks) == 1
    scen = list(range(len(case.scenarios))) if scen is None else list(scen)
    nb = len(scen)
    net = case.networks[0]
    K = net.K
    # per-scenario pieces
    pieces = []
    for s in scen:
        qp = D.assemble(case, s, net.eta_min)   # bounds replaced below
        w = case.scenarios[s].weight / nb
        # a bound a_i eta_j with a_i = 0 (no availability) is a static bound
        up = (qp.hi_idx >= 0) & (qp.hi_coef != 0)
        lw = (qp.lo_idx >= 0) & (qp.lo_coef != 0)
        pieces.append((qp, w, np.where(up)[0], np.where(lw)[0]))
    # assemble: vars = [eta | x_1 s^u_1 s^l_1 | x_2 ...]
    cols = K
    layout = []
    for qp, w, up, lw in pieces:
        layout.append((cols, qp.n, len(up), len(lw)))
        cols += qp.n + len(up) + len(lw)
    nvar = cols
    rows, cc, vals, rhs = [], [], [], []
    nrow = 0
    q = np.zeros(nvar)
    Qd = np.zeros(nvar)
    lo = np.zeros(nvar)
    hi = np.full(nvar, np.inf)
    q[:K] = net.gamma
    lo[:K] = net.eta_min
    hi[:K] = net.eta_max
    for (qp, w, up, lw), (c0, n, nu, nl) in zip(pieces, layout):
        Ec = qp.E.tocoo()
        rows.append(Ec.row + nrow)
        cc.append(Ec.col + c0)
        vals.append(Ec.data)
        rhs.append(qp.e)
        nrow += qp.m
        q[c0:c0 + n] = w * qp.q
        Qd[c0:c0 + n] = w * qp.r
        # static bounds of x: keep the finite bound that does not depend on eta
        dep_up = np.zeros(n, bool)
        dep_up[up] = True
        dep_lw = np.zeros(n, bool)
        dep_lw[lw] = True
        xlo = np.where(dep_lw, -np.inf, np.where(qp.lo_idx >= 0, 0.0, qp.lo))
        xhi = np.where(dep_up, np.inf, np.where(qp.hi_idx >= 0, 0.0, qp.hi))
        lo[c0:c0 + n] = xlo
        hi[c0:c0 + n] = xhi
        # x_i + s_i - a_i eta_j = 0
        su = c0 + n + np.arange(nu)
        r = nrow + np.arange(nu)
        rows += [r, r, r]
        cc += [c0 + up, su, qp.hi_idx[up]]
        vals += [np.ones(nu), np.ones(nu), -qp.hi_coef[up]]
        rhs.append(np.zeros(nu))
        nrow += nu
        # x_i - s_i - a_i eta_j = 0   (x_i >= a_i eta_j)
        sl = c0 + n + nu + np.arange(nl)
        r = nrow + np.arange(nl)
        rows += [r, r, r]
        cc += [c0 + lw, sl, qp.lo_idx[lw]]
        vals += [np.ones(nl), -np.ones(nl), -qp.lo_coef[lw]]
        rhs.append(np.zeros(nl))
        nrow += nl
        lo[su] = 0.0
        lo[sl] = 0.0
    E = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cc))), shape=(nrow, nvar))
    e = np.concatenate(rhs)
    jqp = D.QP(E=E, e=e, q=q, lo=lo, hi=hi, r=0.0, hi_idx=np.full(nvar, -1), hi_coef=np.zeros(nvar),
               lo_idx=np.full(nvar, -1), lo_coef=np.zeros(nvar), emis=np.zeros(nvar), fuel=np.zeros(nvar),
               dims={}, K=K)
    sol = D.solve_ipm(jqp, tol=1e-10, max_iter=300, qdiag=Qd)
    eta = np.clip(sol.x[:K], net.eta_min, net.eta_max)
    val = float(0.5 * np.dot(Qd * sol.x, sol.x) + q @ sol.x)
    return eta, val, sol.status
