"""FP64 oracle for one scenario's economic dispatch (the dispatch map).

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
GPU path.

Section 2.1 of the paper defines the dispatch map x*_s(eta) as the minimiser of
an operating cost c_s(x) subject to constraints A_s(eta) x <= b_s(eta) whose
right-hand side depends on the capacities (e.g. a generator's power limit
depends on its capacity entry).  The paper leaves the device models to its
companion work; this oracle fixes them as follows (one scenario, hours
t = 0..T-1, 1 h steps):

variables (canonical order, each block [device][hour])
    p   [G,T]  generator output            0 <= p <= avail[g,t] * eta_g
    f   [L,T]  line flow, from -> to        -eta_l <= f <= eta_l
               (the last n_hvdc lines are HVDC links, the rest AC lines)
    th  [N,T]  bus voltage angle            free
    ch  [B,T]  battery charge               0 <= ch <= eta_k
    dis [B,T]  battery discharge            0 <= dis <= eta_k
    soc [B,T]  battery state of charge      0 <= soc <= H * eta_k
    u   [N,T]  unserved load                u >= 0
    s   [R,T]  ramp of a ramp-limited generator g_r between hours t-1 and t,
               -rho_g eta_g <= s <= rho_g eta_g  (rho_g: the share of its
               capacity a unit can move in an hour; units without a limit
               have no ramp variables)

equalities (canonical order; duals y = [pi | mu | nu])
    balance [N,T]: sum_{g at n} p + sum_{k at n} (dis - ch) + u
                   + sum_{l: to(l)=n} f - sum_{l: from(l)=n} f = D[n,t]
    flow    [L_ac,T]: f - beta_l (th[from(l)] - th[to(l)]) = 0  (DC power flow,
                   AC lines l < L_ac only; an HVDC link's flow is a free
                   transfer within its capacity, so it enters the two
                   balance rows and nothing else).  On a network whose
                   susceptances scale with capacity (Section 2.1's A_s(eta):
                   an expanded line is parallel circuits of the same kind)
                   beta_l = line_beta_l * eta_l / eta_min_l.
    soc     [B,T]: soc[t] - soc[t-1] - eff * ch[t] + dis[t] = 0, cyclic in t
    ramp    [R,T]: p[g_r,t] - p[g_r,t-1] - s[r,t] = 0, cyclic in t

objective
    c(x) = sum c_g p + lambda_u sum u + (r/2) ||x||^2

i.e. the standard form  min (r/2)||x||^2 + q'x  s.t.  E x = e,  l <= x <= u,
with Lagrangian  (r/2)||x||^2 + q'x - y'(E x - e).  The multiplier of a box
is  z = E'y - q - r x  (z >= 0 at an upper bound, z <= 0 at a lower bound,
z = 0 for a free entry), so pi is the locational marginal price.

The solve is a textbook Mehrotra predictor-corrector primal-dual interior
point method for convex QPs with equality constraints and simple bounds
(Nocedal & Wright, Numerical Optimization, 2nd ed., Sec. 16.6; Wright,
Primal-Dual Interior-Point Methods, 1997), followed by an exact active-set
polish.  Each Newton step reduces to the sparse SPD normal system
E H^-1 E', factorised with SuperLU.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

INF = np.inf


@dataclasses.dataclass
class QP:
    """One scenario's dispatch QP in standard form plus the map from bounds
    to capacity entries (used by the gradient)."""
    E: sp.csr_matrix
    e: np.ndarray
    q: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    r: float
    # bound -> capacity map: for entry i, hi_i = hi_coef[i] * eta[hi_idx[i]]
    # when hi_idx[i] >= 0 (likewise lo); indices are local to the network
    hi_idx: np.ndarray
    hi_coef: np.ndarray
    lo_idx: np.ndarray
    lo_coef: np.ndarray
    emis: np.ndarray          # t/MWh per variable (generators only)
    fuel: np.ndarray          # $/MWh per variable excluding the unserved penalty
    dims: dict                # block sizes
    K: int
    # d beta_l / d eta_l per line (0 where beta does not depend on eta):
    # the constraint matrix's dependence on the capacities
    line_dbeta: Optional[np.ndarray] = None

    @property
    def n(self):
        return self.E.shape[1]

    @property
    def m(self):
        return self.E.shape[0]


def block_slices(G, L, N, B, T, R=0):
    """Canonical variable blocks (the ordering both sides agree on)."""
    sizes = [("p", G), ("f", L), ("th", N), ("ch", B), ("dis", B), ("soc", B), ("u", N), ("s", R)]
    out, o = {}, 0
    for name, c in sizes:
        out[name] = slice(o, o + c * T)
        o += c * T
    out["n"] = o
    return out


def row_slices(N, L, B, T, R=0):
    out, o = {}, 0
    for name, c in [("bal", N), ("flow", L), ("soc", B), ("ramp", R)]:
        out[name] = slice(o, o + c * T)
        o += c * T
    out["m"] = o
    return out


def assemble(case, s: int, eta_net: np.ndarray) -> QP:
    """Build scenario ``s``'s dispatch QP at the network's capacities
    ``eta_net`` = [generators | lines | batteries] (Section 2.1, eq. (2))."""
    sc = case.scenarios[s]
    net = case.networks[sc.network]
    G, L, N, B, T = net.n_gens, net.n_lines, net.n_nodes, net.n_batt, sc.T
    Lac = L - int(getattr(net, "n_hvdc", 0))
    ramp = getattr(net, "gen_ramp", None)
    rg = np.zeros(0, np.int64) if ramp is None else np.where(np.asarray(ramp) > 0)[0]
    R = rg.shape[0]
    K = net.K
    eta_net = np.asarray(eta_net, dtype=np.float64)
    assert eta_net.shape == (K,)
    vs = block_slices(G, L, N, B, T, R)
    rs = row_slices(N, Lac, B, T, R)
    n, m = vs["n"], rs["m"]
    t = np.arange(T)

    def vidx(block, dev):       # variable index of (dev, t) pairs, shape [len(dev), T]
        return vs[block].start + np.asarray(dev)[:, None] * T + t[None, :]

    def ridx(block, dev):
        return rs[block].start + np.asarray(dev)[:, None] * T + t[None, :]

    rows, cols, vals = [], [], []

    def put(r, c, v):
        r, c = np.broadcast_arrays(r, c)
        rows.append(r.ravel())
        cols.append(c.ravel())
        vals.append(np.broadcast_to(v, r.shape).ravel().astype(np.float64))

    # balance rows
    put(ridx("bal", net.gen_node), vidx("p", np.arange(G)), 1.0)
    put(ridx("bal", net.batt_node), vidx("dis", np.arange(B)), 1.0)
    put(ridx("bal", net.batt_node), vidx("ch", np.arange(B)), -1.0)
    put(ridx("bal", np.arange(N)), vidx("u", np.arange(N)), 1.0)
    put(ridx("bal", net.line_to), vidx("f", np.arange(L)), 1.0)
    put(ridx("bal", net.line_from), vidx("f", np.arange(L)), -1.0)
    # flow rows of the AC lines: f - beta (th_from - th_to) = 0
    ac = np.arange(Lac)
    beta = np.asarray(net.line_beta[:Lac], np.float64)
    dbeta = np.zeros(L)
    if getattr(net, "beta_scales", False):
        ref = np.asarray(net.eta_min[G:G + Lac], np.float64)
        dbeta[:Lac] = beta / ref
        beta = beta * eta_net[G:G + Lac] / ref
    put(ridx("flow", ac), vidx("f", ac), 1.0)
    put(ridx("flow", ac), vidx("th", net.line_from[:Lac]), -beta[:, None])
    put(ridx("flow", ac), vidx("th", net.line_to[:Lac]), beta[:, None])
    # soc rows: soc[t] - soc[t-1] - eff ch[t] + dis[t] = 0 (cyclic)
    kb = np.arange(B)
    put(ridx("soc", kb), vidx("soc", kb), 1.0)
    prev = vs["soc"].start + kb[:, None] * T + ((t - 1) % T)[None, :]
    put(ridx("soc", kb), prev, -1.0)
    put(ridx("soc", kb), vidx("ch", kb), -case.eff)
    put(ridx("soc", kb), vidx("dis", kb), 1.0)
    # ramp rows: p[g, t] - p[g, t-1] - s[r, t] = 0 (cyclic)
    if R:
        rr = np.arange(R)
        put(ridx("ramp", rr), vidx("p", rg), 1.0)
        put(ridx("ramp", rr), vs["p"].start + rg[:, None] * T + ((t - 1) % T)[None, :], -1.0)
        put(ridx("ramp", rr), vidx("s", rr), -1.0)

    E = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m, n))
    E.sum_duplicates()
    if T == 1 and (B > 0 or R > 0):
        # soc[t] - soc[t-1] and p[t] - p[t-1] cancel when T == 1; drop explicit zeros
        E.eliminate_zeros()

    e = np.zeros(m)
    e[rs["bal"]] = sc.load.ravel()

    q = np.zeros(n)
    q[vs["p"]] = np.repeat(net.gen_cost, T)
    q[vs["u"]] = case.lambda_u
    fuel = np.zeros(n)
    fuel[vs["p"]] = np.repeat(net.gen_cost, T)
    emis = np.zeros(n)
    emis[vs["p"]] = np.repeat(net.gen_emis, T)

    lo = np.zeros(n)
    hi = np.full(n, INF)
    hi_idx = np.full(n, -1, dtype=np.int64)
    lo_idx = np.full(n, -1, dtype=np.int64)
    hi_coef = np.zeros(n)
    lo_coef = np.zeros(n)

    eg = eta_net[:G]
    el = eta_net[G:G + L]
    eb = eta_net[G + L:]
    hi[vs["p"]] = (sc.avail * eg[:, None]).ravel()
    hi_idx[vs["p"]] = np.repeat(np.arange(G), T)
    hi_coef[vs["p"]] = sc.avail.ravel()

    hi[vs["f"]] = np.repeat(el, T)
    lo[vs["f"]] = -np.repeat(el, T)
    hi_idx[vs["f"]] = np.repeat(G + np.arange(L), T)
    lo_idx[vs["f"]] = np.repeat(G + np.arange(L), T)
    hi_coef[vs["f"]] = 1.0
    lo_coef[vs["f"]] = -1.0

    lo[vs["th"]] = -INF

    for blk, mult in (("ch", 1.0), ("dis", 1.0), ("soc", case.hours)):
        hi[vs[blk]] = mult * np.repeat(eb, T)
        hi_idx[vs[blk]] = np.repeat(G + L + np.arange(B), T)
        hi_coef[vs[blk]] = mult

    if R:
        rho = np.asarray(ramp, np.float64)[rg]
        hi[vs["s"]] = np.repeat(rho * eg[rg], T)
        lo[vs["s"]] = -np.repeat(rho * eg[rg], T)
        hi_idx[vs["s"]] = np.repeat(rg, T)
        lo_idx[vs["s"]] = np.repeat(rg, T)
        hi_coef[vs["s"]] = np.repeat(rho, T)
        lo_coef[vs["s"]] = -np.repeat(rho, T)

    return QP(E=E, e=e, q=q, lo=lo, hi=hi, r=float(case.r), hi_idx=hi_idx, hi_coef=hi_coef,
              lo_idx=lo_idx, lo_coef=lo_coef, emis=emis, fuel=fuel,
              dims=dict(G=G, L=L, Lac=Lac, N=N, B=B, T=T, R=R, ramp_gen=rg, vs=vs, rs=rs,
                        line_from=np.asarray(net.line_from), line_to=np.asarray(net.line_to)), K=K,
              line_dbeta=dbeta if dbeta.any() else None)


# --------------------------------------------------------------------------
# objective, dual function and the solver-independent KKT residual
# --------------------------------------------------------------------------

def primal_objective(qp: QP, x: np.ndarray) -> float:
    """c(x) = (r/2)||x||^2 + q'x."""
    return float(0.5 * qp.r * np.dot(x, x) + np.dot(qp.q, x))


def lagrangian_minimiser(qp: QP, y: np.ndarray) -> np.ndarray:
    """argmin over the box of (r/2)||x||^2 + q'x - y'E x; closed form because
    the Hessian is r I and every inequality is a box."""
    return np.clip((qp.E.T @ y - qp.q) / qp.r, qp.lo, qp.hi)


def dual_function(qp: QP, y: np.ndarray) -> float:
    """Exact dual function D(y) = min_{lo<=x<=hi} L(x, y); a lower bound on the
    optimal value for every y (r > 0, so it is finite everywhere)."""
    xy = lagrangian_minimiser(qp, y)
    ety = qp.E.T @ y
    return float(np.dot(qp.q, xy) + 0.5 * qp.r * np.dot(xy, xy) - np.dot(ety, xy) + np.dot(qp.e, y))


def kkt_residual(qp: QP, x: np.ndarray, y: np.ndarray) -> dict:
    """Solver-independent relative KKT residual of a pair (x, y):

    r_pri = ||E x - e||_inf / (1 + ||e||_inf)
    r_dual = ||(E'y - q - r x)_free||_inf / (1 + ||q||_inf) over entries with
             no finite bound (the angles); boxed entries carry no dual
             feasibility condition because their multipliers are implicit in D
    r_gap = |P(x) - D(y)| / (1 + max(|P(x)|, |D(y)|))
    r_box = largest bound violation of x relative to (1 + ||bounds||_inf)

    ``kkt`` is the max of the four.  All are zero exactly at an optimal pair.
    """
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    rp = qp.E @ x - qp.e
    r_pri = float(np.abs(rp).max(initial=0.0) / (1.0 + np.abs(qp.e).max(initial=0.0)))
    free = np.isinf(qp.lo) & np.isinf(qp.hi)
    zd = qp.E.T @ y - qp.q - qp.r * x
    r_dual = float(np.abs(zd[free]).max(initial=0.0) / (1.0 + np.abs(qp.q).max(initial=0.0)))
    P = primal_objective(qp, x)
    D = dual_function(qp, y)
    r_gap = abs(P - D) / (1.0 + max(abs(P), abs(D)))
    bmag = max(np.abs(qp.lo[np.isfinite(qp.lo)]).max(initial=0.0),
               np.abs(qp.hi[np.isfinite(qp.hi)]).max(initial=0.0))
    viol = np.maximum(qp.lo - x, x - qp.hi)
    viol = viol[np.isfinite(viol)]
    r_box = float(max(0.0, viol.max(initial=0.0)) / (1.0 + bmag))
    return dict(r_pri=r_pri, r_dual=r_dual, r_gap=float(r_gap), r_box=r_box,
                kkt=max(r_pri, r_dual, float(r_gap), r_box), P=P, D=D)


# --------------------------------------------------------------------------
# interior point
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Solution:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray             # box multipliers E'y - q - r x
    obj: float
    iters: int
    status: str
    history: list             # per-iteration (KKT residual, seconds) of the iterate when tracked
    polished: bool = False
    degenerate: bool = False  # weakly active bounds or rank-deficient E_F
    active_lo: Optional[np.ndarray] = None
    active_hi: Optional[np.ndarray] = None


def _normal_solve(E, hinv, rhs, reg=0.0):
    M = (E @ sp.diags(hinv) @ E.T).tocsc()
    if reg > 0:
        M = M + reg * sp.identity(M.shape[0], format="csc")
    lu = spla.splu(M, permc_spec="MMD_AT_PLUS_A", options=dict(SymmetricMode=True))
    return lu


def solve_ipm(qp: QP, tol: float = 1e-10, max_iter: int = 200, track: bool = False,
              qdiag: Optional[np.ndarray] = None) -> Solution:
    """Mehrotra predictor-corrector for min 0.5 x'Qx + q'x, E x = e,
    lo <= x <= hi, with Q = diag(qdiag) (default r I).  Entries with
    lo == hi are fixed and eliminated; free and one-sided bounds are
    allowed.  ``track`` records the solver-independent KKT residual of each
    iterate and the wall time (perf_counter) at which it was reached, as
    (kkt, seconds since the start) pairs (used to time when 1e-4 is first
    reached)."""
    t_start = time.perf_counter()
    n, m = qp.n, qp.m
    Qd = np.full(n, qp.r) if qdiag is None else np.asarray(qdiag, np.float64)
    fixed = np.isfinite(qp.lo) & np.isfinite(qp.hi) & (qp.hi - qp.lo <= 1e-12 * (1 + np.abs(qp.hi)))
    act = ~fixed
    E_full = qp.E.tocsc()
    Ea = E_full[:, act].tocsr()
    xfix = np.where(fixed, qp.lo, 0.0)
    e = qp.e - E_full @ xfix
    q = qp.q[act]
    Q = Qd[act]
    lo = qp.lo[act]
    hi = qp.hi[act]
    hasl = np.isfinite(lo)
    hasu = np.isfinite(hi)
    na = int(act.sum())

    # starting point: interior, scaled to the bounds
    x = np.zeros(na)
    both = hasl & hasu
    x[both] = 0.5 * (lo[both] + hi[both])
    x[hasl & ~hasu] = lo[hasl & ~hasu] + 1.0
    x[~hasl & hasu] = hi[~hasl & hasu] - 1.0
    zscale = max(1.0, float(np.abs(q).max(initial=0.0)) * 1e-2)
    zl = np.where(hasl, zscale, 0.0)
    zu = np.where(hasu, zscale, 0.0)
    y = np.zeros(m)
    nb = int(hasl.sum() + hasu.sum())
    enorm = 1.0 + np.abs(e).max(initial=0.0)
    qnorm = 1.0 + np.abs(q).max(initial=0.0)
    hist = []
    status = "max_iter"
    it = 0
    for it in range(1, max_iter + 1):
        sl = np.where(hasl, x - lo, 1.0)
        su = np.where(hasu, hi - x, 1.0)
        rd = Q * x + q - Ea.T @ y - zl + zu
        rp = Ea @ x - e
        mu = (np.dot(sl[hasl], zl[hasl]) + np.dot(su[hasu], zu[hasu])) / max(nb, 1)
        P = 0.5 * np.dot(Q * x, x) + np.dot(q, x)
        if track:
            xf = np.where(fixed, qp.lo, 0.0)
            xf[act] = x
            hist.append((kkt_residual(qp, xf, y)["kkt"], time.perf_counter() - t_start))
        if (np.abs(rp).max(initial=0.0) / enorm < tol and np.abs(rd).max(initial=0.0) / qnorm < tol
                and mu * max(nb, 1) / (1.0 + abs(P)) < tol):
            status = "optimal"
            break
        H = Q + np.where(hasl, zl / sl, 0.0) + np.where(hasu, zu / su, 0.0)
        hinv = 1.0 / H
        try:
            lu = _normal_solve(Ea, hinv, None)
        except RuntimeError:
            lu = _normal_solve(Ea, hinv, None, reg=1e-12 * float(hinv.max()))

        def newton(rcl, rcu):
            rhsx = -rd + np.where(hasl, rcl / sl, 0.0) - np.where(hasu, rcu / su, 0.0)
            dy = lu.solve(-rp - Ea @ (hinv * rhsx))
            dx = hinv * (rhsx + Ea.T @ dy)
            dzl = np.where(hasl, (rcl - zl * dx) / sl, 0.0)
            dzu = np.where(hasu, (rcu + zu * dx) / su, 0.0)
            return dx, dy, dzl, dzu

        def steplen(dx, dzl, dzu):
            a = 1.0
            with np.errstate(divide="ignore", invalid="ignore"):
                m1 = hasl & (dx < 0)
                if m1.any():
                    a = min(a, float(np.min(-sl[m1] / dx[m1])))
                m2 = hasu & (dx > 0)
                if m2.any():
                    a = min(a, float(np.min(su[m2] / dx[m2])))
                m3 = hasl & (dzl < 0)
                if m3.any():
                    a = min(a, float(np.min(-zl[m3] / dzl[m3])))
                m4 = hasu & (dzu < 0)
                if m4.any():
                    a = min(a, float(np.min(-zu[m4] / dzu[m4])))
            return a

        # predictor (affine scaling)
        rcl = np.where(hasl, -sl * zl, 0.0)
        rcu = np.where(hasu, -su * zu, 0.0)
        dxa, dya, dzla, dzua = newton(rcl, rcu)
        aa = steplen(dxa, dzla, dzua)
        sl_a = sl + aa * dxa
        su_a = su - aa * dxa
        mu_a = (np.dot(sl_a[hasl], (zl + aa * dzla)[hasl]) +
                np.dot(su_a[hasu], (zu + aa * dzua)[hasu])) / max(nb, 1)
        sigma = (mu_a / mu) ** 3 if mu > 0 else 0.0
        # corrector with centring
        rcl = np.where(hasl, -sl * zl - dxa * dzla + sigma * mu, 0.0)
        rcu = np.where(hasu, -su * zu + dxa * dzua + sigma * mu, 0.0)
        dx, dy, dzl, dzu = newton(rcl, rcu)
        a = min(1.0, 0.995 * steplen(dx, dzl, dzu))
        x = x + a * dx
        y = y + a * dy
        zl = zl + a * dzl
        zu = zu + a * dzu
    xf = np.where(fixed, qp.lo, 0.0)
    xf[act] = x
    z = qp.E.T @ y - qp.q - qp.r * xf if qdiag is None else qp.E.T @ y - qp.q - Qd * xf
    sol = Solution(x=xf, y=y, z=z, obj=primal_objective(qp, xf) if qdiag is None else
                   float(0.5 * np.dot(Qd * xf, xf) + np.dot(qp.q, xf)),
                   iters=it, status=status, history=hist)
    # keep the interior-point complementarity information for polishing
    sol._ipm = dict(act=act, fixed=fixed, zl=zl, zu=zu, x=x)
    return sol


def _free_factor(qp: QP, free: np.ndarray):
    E = qp.E.tocsc()
    EF = E[:, free].tocsr()
    EA = E[:, ~free]
    M = (EF @ EF.T).tocsc()
    rowsum = np.asarray(np.abs(EF).sum(axis=1)).ravel()
    scale = float(M.diagonal().max(initial=1.0))
    Mr = M + 1e-13 * scale * sp.identity(M.shape[0], format="csc")
    lu = spla.splu(Mr, permc_spec="MMD_AT_PLUS_A", options=dict(SymmetricMode=True))

    def solve(b):
        v = lu.solve(b)
        for _ in range(3):   # iterative refinement on the regularised system
            v = v + lu.solve(b - M @ v)
        return v
    return EF, EA, solve, bool((rowsum == 0).any())


def _reduced_solve(qp: QP, free: np.ndarray, xA: np.ndarray, y0: np.ndarray):
    """Equality-constrained solve on the free set F with the active entries
    fixed at ``xA`` (a full-length vector, used where ~free):
    r x_F + q_F = E_F' y,  E_F x_F = e - E_A x_A.

    x_F is unique; y is unique only when E_F has full row rank.  The returned
    y is the multiplier closest to ``y0`` (the interior-point dual, which sits
    in the relative interior of the optimal dual face), so degenerate rows keep
    a valid multiplier.  Returns (x, y, rank_deficient)."""
    EF, EA, msolve, rankdef = _free_factor(qp, free)
    b = qp.r * (qp.e - EA @ xA[~free]) + EF @ qp.q[free]
    yt = msolve(b)
    x = xA.copy()
    x[free] = (EF.T @ yt - qp.q[free]) / qp.r
    g = qp.r * x[free] + qp.q[free] - EF.T @ y0
    y = y0 + msolve(EF @ g)
    return x, y, rankdef


def adjoint_lsq(qp: QP, free: np.ndarray, g: np.ndarray):
    """Least-squares adjoint  w = argmin ||E_F' w - g_F||  (normal equations
    E_F E_F' w = E_F g_F).  Returns (w, rank_deficient)."""
    EF, EA, msolve, rankdef = _free_factor(qp, free)
    return msolve(EF @ g[free]), rankdef


def polish(qp: QP, sol: Solution, tol_act: float = 1e-9, max_rounds: int = 60) -> Solution:
    """Exact active-set polish.

    Bounds are first classified from the interior-point complementarity pairs
    (an entry is active when its multiplier exceeds its slack).  The active
    entries are fixed at their bounds and the remaining equality QP is solved
    with a sparse direct solve.  Entries that leave their box are then moved
    to the violated bound and active entries whose multiplier has the wrong
    sign are released (a primal-dual active-set iteration), until the
    classification is stable.  The result is accepted when it is primal
    feasible and every multiplier has the right sign."""
    info = sol._ipm
    act, fixed, zl, zu = info["act"], info["fixed"], info["zl"], info["zu"]
    lo, hi = qp.lo, qp.hi
    x = sol.x
    n = qp.n
    zl_f = np.zeros(n)
    zu_f = np.zeros(n)
    zl_f[act] = zl
    zu_f[act] = zu
    sl = np.where(np.isfinite(lo), x - lo, INF)
    su = np.where(np.isfinite(hi), hi - x, INF)
    at_lo = (np.isfinite(lo) & (zl_f > sl) & ~fixed) | fixed
    at_hi = np.isfinite(hi) & (zu_f > su) & ~at_lo
    ipm_lo, ipm_hi = at_lo.copy(), at_hi.copy()
    bscale = 1.0 + np.abs(qp.q).max()
    xs = 1.0 + max(np.abs(lo[np.isfinite(lo)]).max(initial=0), np.abs(hi[np.isfinite(hi)]).max(initial=0))
    ok = False
    y0 = sol.y
    for _ in range(max_rounds):
        free = ~(at_lo | at_hi)
        xA = np.where(at_lo, lo, np.where(at_hi, hi, 0.0))
        xp, yp, rankdef = _reduced_solve(qp, free, xA, y0)
        z = qp.E.T @ yp - qp.q - qp.r * xp
        below = free & (xp < lo - 1e-10 * xs)
        above = free & (xp > hi + 1e-10 * xs)
        wrong_hi = at_hi & ~fixed & (z < -1e-9 * bscale)
        wrong_lo = at_lo & ~fixed & (z > 1e-9 * bscale)
        if not (below.any() or above.any() or wrong_hi.any() or wrong_lo.any()):
            resid = np.abs(qp.E @ xp - qp.e)
            bad = resid > 1e-8 * (1 + np.abs(qp.e).max(initial=0))
            if not bad.any():
                ok = True
                break
            # rows the active set makes unsatisfiable (a weakly active entry
            # was classified active): release the active entry of those rows
            # with the smallest multiplier
            touch = np.asarray(np.abs(qp.E[bad]).sum(axis=0)).ravel() > 0
            cand = np.where(touch & (at_lo | at_hi) & ~fixed)[0]
            if cand.size == 0:
                break
            j = cand[np.argmin(np.abs(z[cand]))]
            at_lo[j] = False
            at_hi[j] = False
            y0 = yp
            continue
        at_lo = (at_lo & ~wrong_lo) | below
        at_hi = (at_hi & ~wrong_hi) | above
        y0 = yp
    weak = (np.abs(z[(at_lo | at_hi) & ~fixed]) < tol_act * bscale).any()
    out = dataclasses.replace(sol)
    out._ipm = sol._ipm
    if ok:
        out.x, out.y, out.z = np.clip(xp, lo, hi), yp, z
        out.obj = primal_objective(qp, out.x)
        out.polished = True
        out.active_lo = at_lo
        out.active_hi = at_hi
    else:
        # the refinement did not settle: a weakly active entry (slack and
        # multiplier both near zero) sits at a kink of the dispatch map; keep
        # the interior-point solution and its classification
        out.active_lo = ipm_lo
        out.active_hi = ipm_hi
        weak = True
    out.degenerate = bool(weak or rankdef)
    return out


def solve(qp: QP, tol: float = 1e-10, do_polish: bool = True, track: bool = False) -> Solution:
    sol = solve_ipm(qp, tol=tol, track=track)
    if do_polish:
        sol = polish(qp, sol)
    return sol


def solve_scenario(case, s: int, eta: np.ndarray, **kw):
    """Solve scenario s at the case-wide capacity vector ``eta``."""
    off = case.eta_offsets()
    net_id = case.scenarios[s].network
    qp = assemble(case, s, np.asarray(eta)[off[net_id]:off[net_id + 1]])
    return qp, solve(qp, **kw)


def operating_cost(qp: QP, x: np.ndarray) -> float:
    """c_s(x): fuel + unserved penalty + regulariser."""
    return primal_objective(qp, x)


def planner_objective(qp: QP, x: np.ndarray, omega: float, y: Optional[np.ndarray] = None,
                      lmp: float = 0.0) -> float:
    """h_s = c_s(x) + omega * emissions(x) (emissions-aware planning,
    Section 2.1) + lmp * sum_{n,t} pi[n,t] D[n,t] (a planner objective built
    on the locational marginal prices, Section 2.1: what consumers pay at
    those prices; y the duals, whose balance block is pi)."""
    h = primal_objective(qp, x) + omega * float(np.dot(qp.emis, x))
    if lmp:
        rs = qp.dims["rs"]["bal"]
        h += lmp * float(np.dot(qp.e[rs], y[rs]))
    return h
