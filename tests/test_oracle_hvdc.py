"""Pins for HVDC links in the oracle (Section 3.1's case mixes AC lines and
HVDC links; Section 2.1 eq. (2) with a link's flow bounded by its capacity).

An HVDC link carries a flow chosen freely within [-eta, eta]: it enters the
balance rows of its two nodes and no power-flow row, so no angle is tied to
it.  The closed forms below follow from the dispatch KKT conditions with the
quadratic regulariser r on every variable."""
import numpy as np
import pytest

from paper_2410_13055_amd import cases
from oracle import dispatch as D
from oracle import gradient as Gm


def _solve(case, eta=None, s=0):
    eta = case.eta_min() if eta is None else eta
    return D.solve_scenario(case, s, eta)


@pytest.mark.parametrize("cA,cB,D_,F", [(20.0, 60.0, 150.0, 80.0), (35.0, 75.0, 210.0, 130.0)])
def test_hvdc_two_node_congested_closed_form(cA, cB, D_, F):
    # the link is full: p_A = f = F, p_B = D - F; no angle is tied to the
    # flow, so both angles sit at the regulariser's minimum, zero
    cs = cases.hvdc_two_node(cA=cA, cB=cB, D=D_, F=F)
    qp, sol = _solve(cs)
    r = cs.r
    vs, rs = qp.dims["vs"], qp.dims["rs"]
    x = sol.x
    assert qp.m == 2 and qp.dims["Lac"] == 0     # two balance rows, no flow row
    np.testing.assert_allclose(x[vs["p"]], [F, D_ - F], atol=1e-7)
    np.testing.assert_allclose(x[vs["f"]], [F], atol=1e-7)
    np.testing.assert_allclose(x[vs["th"]], 0.0, atol=1e-12)
    np.testing.assert_allclose(x[vs["u"]], 0.0, atol=1e-7)
    np.testing.assert_allclose(sol.y[rs["bal"]], [cA + r * F, cB + r * (D_ - F)], rtol=1e-9)
    V = cA * F + cB * (D_ - F) + 0.5 * r * (2 * F ** 2 + (D_ - F) ** 2)
    assert abs(sol.obj - V) <= 1e-9 * V
    # d/dF of V along the binding bound: cA - cB + r (F - (D - F) + F)
    gr = Gm.scenario_gradient(qp, sol, 0.0)
    np.testing.assert_allclose(gr["grad"], [0.0, 0.0, cA - cB + r * (3 * F - D_)], atol=1e-7)


def test_hvdc_two_node_interior_flow_closed_form():
    # a link wide enough to stay slack: stationarity of the flow gives
    # pi_B - pi_A = r f with pi_A = cA + r f and pi_B = cB + r (D - f), so
    # f = (cB - cA + r D) / (3 r)
    cs = cases.hvdc_two_node(cA=20.0, cB=20.0625, D=150.0, F=100.0)
    net = cs.networks[0]
    cA, cB = net.gen_cost
    r, D_ = cs.r, 150.0
    f = (cB - cA + r * D_) / (3 * r)
    assert 0 < f < 100.0
    qp, sol = _solve(cs)
    vs = qp.dims["vs"]
    np.testing.assert_allclose(sol.x[vs["f"]], [f], atol=1e-6)
    np.testing.assert_allclose(sol.x[vs["p"]], [f, D_ - f], atol=1e-6)
    np.testing.assert_allclose(sol.x[vs["th"]], 0.0, atol=1e-12)
    gr = Gm.scenario_gradient(qp, sol, 0.0)
    np.testing.assert_allclose(gr["grad"], 0.0, atol=1e-9)


def test_hvdc_differs_from_the_same_ac_line():
    # the AC line's flow also pays the angle regulariser (f = beta dtheta),
    # so at equal data the AC optimum moves less power than the link
    ac = cases.two_node(cA=20.0, cB=20.0625, D=150.0, F=100.0, beta=0.05)
    dc = cases.hvdc_two_node(cA=20.0, cB=20.0625, D=150.0, F=100.0)
    qa, sa = _solve(ac)
    qd, sd = _solve(dc)
    assert qa.m == qd.m + 1
    fa, fd = sa.x[qa.dims["vs"]["f"]][0], sd.x[qd.dims["vs"]["f"]][0]
    assert fa < fd - 1.0
    assert np.abs(sa.x[qa.dims["vs"]["th"]]).max() > 1.0


def _mixed():
    # links of 5 MW at the lower bound of their box, so they bind
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=2, seed=7, n_hvdc=2)
    net = cs.networks[0]
    net.eta_min[net.n_gens + net.n_ac:net.n_gens + net.n_lines] = 5.0
    return cs


def test_mixed_network_rows_and_physics():
    cs = _mixed()
    net = cs.networks[0]
    assert net.n_hvdc == 2 and net.n_ac == net.n_lines - 2
    # the AC part of the case is the one without links
    base = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=2, seed=7)
    np.testing.assert_array_equal(net.line_from[:net.n_ac], base.networks[0].line_from)
    np.testing.assert_array_equal(cs.scenarios[1].load, base.scenarios[1].load)
    qp, sol = _solve(cs, s=1)
    d = qp.dims
    T, N, B = d["T"], d["N"], d["B"]
    assert qp.m == (N + net.n_ac + B) * T
    E = qp.E.tocsc()
    for l in range(net.n_ac, net.n_lines):     # each link's flow: two balance rows, +1 at 'to', -1 at 'from'
        for t in (0, T - 1):
            col = E[:, d["vs"]["f"].start + l * T + t]
            assert col.nnz == 2
            rows = sorted(zip(col.indices.tolist(), col.data.tolist()))
            assert rows == sorted([(net.line_to[l] * T + t, 1.0), (net.line_from[l] * T + t, -1.0)])
    x = sol.x
    th = x[d["vs"]["th"]].reshape(N, T)
    f = x[d["vs"]["f"]].reshape(-1, T)
    ac = slice(0, net.n_ac)
    np.testing.assert_allclose(f[ac], net.line_beta[ac, None] * (th[net.line_from[ac]] - th[net.line_to[ac]]),
                               atol=1e-7)
    # the links run at their capacity and carry power their endpoints'
    # angles would not explain
    dc = slice(net.n_ac, net.n_lines)
    np.testing.assert_allclose(np.abs(f[dc]).max(axis=1), 5.0, atol=1e-7)
    gap = np.abs(f[dc] - net.line_beta[dc, None] * (th[net.line_from[dc]] - th[net.line_to[dc]]))
    assert gap.max() > 1.0
    res = D.kkt_residual(qp, sol.x, sol.y)
    assert res["kkt"] <= 1e-9


def test_mixed_network_link_gradient_matches_resolves():
    # the envelope gradient on the link capacities against central
    # differences of full re-solves (h = 0.05 MW), and the active-set
    # differences on every capacity
    cs = _mixed()
    net = cs.networks[0]
    eta = cases.jitter(cs.eta_min(), 3, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    for omega in (0.0, 200.0):
        qp, sol = _solve(cs, eta, s=0)
        gr = Gm.scenario_gradient(qp, sol, omega)["grad"]
        fd = Gm.fixed_set_differences(qp, sol, omega)
        ok = fd["ok"]
        scale = np.abs(gr).max()
        assert np.abs(fd["central"][ok] - gr[ok]).max() <= 1e-6 * scale
        h = 0.05
        assert np.all(gr[net.n_gens + net.n_ac:net.n_gens + net.n_lines] < 0)   # the links bind
        for l in range(net.n_ac, net.n_lines):
            j = net.n_gens + l
            vals = []
            for sgn in (1, -1):
                e2 = eta.copy()
                e2[j] += sgn * h
                q2, s2 = _solve(cs, e2, s=0)
                vals.append(D.planner_objective(q2, s2.x, omega))
            np.testing.assert_allclose((vals[0] - vals[1]) / (2 * h), gr[j], atol=1e-5 * scale)
