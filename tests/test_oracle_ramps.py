"""Pins for generator ramp limits in the oracle (the paper's closing
discussion names ramping limits among the constraints the method keeps): a
ramp-limited unit g moves at most rho_g * eta_g between consecutive hours,
written as rows p[g, t] - p[g, t-1] - s[g, t] = 0 (cyclic in t, like the
battery chains) with the ramp s boxed by the capacity."""
import numpy as np
import pytest

from paper_2410_13055_amd import cases
from oracle import dispatch as D
from oracle import gradient as Gm


def _two_hour(rho=0.2, cA=20.0, cB=60.0, PA=300.0, PB=300.0, D0=100.0, D1=200.0):
    cs = cases.single_node([cA, cB], [PA, PB], np.array([D0, D1]), T=2)
    cs.networks[0].gen_ramp = np.array([rho, 0.0])
    return cs


@pytest.mark.parametrize("rho", [0.2, 0.1])
def test_two_hour_ramp_closed_form(rho):
    # the cheap unit A serves the first hour (load D0) and can only add
    # R = rho PA in the second, the expensive unit B covers the rest:
    # p_A = (D0, D0 + R), p_B = (0, D1 - D0 - R), s = (-R, R); then
    # V(R) = cA (2 D0 + R) + cB (D1 - D0 - R)
    #        + r/2 (D0^2 + (D0 + R)^2 + (D1 - D0 - R)^2 + 2 R^2)
    # and dV/d eta_A = rho dV/dR = rho (cA - cB + r (4R + 2 D0 - D1))
    cA, cB, PA, D0, D1 = 20.0, 60.0, 300.0, 100.0, 200.0
    cs = _two_hour(rho=rho)
    qp, sol = D.solve_scenario(cs, 0, cs.eta_min())
    r, R = cs.r, rho * PA
    vs = qp.dims["vs"]
    assert qp.dims["R"] == 1 and qp.m == 2 + 2        # two balance rows, two ramp rows
    p = sol.x[vs["p"]].reshape(2, 2)
    np.testing.assert_allclose(p[0], [D0, D0 + R], atol=1e-6)
    np.testing.assert_allclose(p[1], [0.0, D1 - D0 - R], atol=1e-6)
    np.testing.assert_allclose(sol.x[vs["s"]], [-R, R], atol=1e-6)
    V = cA * (2 * D0 + R) + cB * (D1 - D0 - R) + 0.5 * r * (D0 ** 2 + (D0 + R) ** 2 + (D1 - D0 - R) ** 2 + 2 * R ** 2)
    assert abs(sol.obj - V) <= 1e-9 * V
    gr = Gm.scenario_gradient(qp, sol, 0.0)
    np.testing.assert_allclose(gr["grad"], [rho * (cA - cB + r * (4 * R + 2 * D0 - D1)), 0.0], atol=1e-7)
    fd = Gm.fixed_set_differences(qp, sol, 0.0)
    assert fd["ok"].all()
    np.testing.assert_allclose(fd["central"], gr["grad"], atol=1e-7)


def test_slack_ramp_changes_nothing():
    # a ramp limit wider than any move the dispatch makes: same point as
    # without it, zero derivative through it
    cs = _two_hour(rho=0.9)
    qp, sol = D.solve_scenario(cs, 0, cs.eta_min())
    base = cases.single_node([20.0, 60.0], [300.0, 300.0], np.array([100.0, 200.0]), T=2)
    qb, sb = D.solve_scenario(base, 0, base.eta_min())
    vs = qp.dims["vs"]
    np.testing.assert_allclose(sol.x[vs["p"]], sb.x[qb.dims["vs"]["p"]], atol=1e-6)
    np.testing.assert_allclose(Gm.scenario_gradient(qp, sol, 0.0)["grad"],
                               Gm.scenario_gradient(qb, sb, 0.0)["grad"], atol=1e-6)


@pytest.mark.parametrize("omega", [0.0, 200.0])
def test_ramped_network_gradient_matches_resolves(omega):
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=1, seed=7, gas_ramp=0.12)
    net = cs.networks[0]
    eta = cases.jitter(cs.eta_min(), 3, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    qp, sol = D.solve_scenario(cs, 0, eta)
    vs = qp.dims["vs"]
    s = sol.x[vs["s"]].reshape(qp.dims["R"], -1)
    lim = (net.gen_ramp[qp.dims["ramp_gen"]] * eta[qp.dims["ramp_gen"]])[:, None]
    assert (np.abs(s) >= lim - 1e-6).any()          # some ramps bind
    gr = Gm.scenario_gradient(qp, sol, omega)["grad"]
    fd = Gm.fixed_set_differences(qp, sol, omega)
    ok = fd["ok"]
    scale = np.abs(gr).max()
    assert np.abs(fd["central"][ok] - gr[ok]).max() <= 1e-6 * scale
    # full re-solves on the ramp-limited units without a kink within h
    h = 1e-3
    js = [j for j in qp.dims["ramp_gen"] if ok[j]][:6]
    assert len(js) == 6
    for j in js:
        vals = []
        for sgn in (1, -1):
            e2 = eta.copy()
            e2[j] += sgn * h
            q2, s2 = D.solve_scenario(cs, 0, e2)
            vals.append(D.planner_objective(q2, s2.x, omega))
        np.testing.assert_allclose((vals[0] - vals[1]) / (2 * h), gr[j], atol=1e-5 * scale)
