"""Pins for a planner objective built on the locational marginal prices
(Section 2.1 lets h_s depend on the LMPs): h = lmp * sum_{n,t} pi[n,t]
D[n,t], what consumers pay at those prices.  Its capacity derivative goes
through the dual solution's sensitivity."""
import numpy as np
import pytest

from paper_2410_13055_amd import cases
from oracle import dispatch as D
from oracle import gradient as Gm


def test_two_load_payments_closed_form():
    # the line is full: p_A = DA + F, p_B = DB - F, so pi_A = cA + r (DA + F)
    # and pi_B = cB + r (DB - F); payments DA pi_A + DB pi_B move with F by
    # r (DA - DB), and with no generator capacity binding that is all
    cA, cB, DA, DB, F = 20.0, 60.0, 50.0, 150.0, 80.0
    cs = cases.two_loads(300.0, 200.0, F, DA=DA, DB=DB, cA=cA, cB=cB)
    qp, sol = D.solve_scenario(cs, 0, cs.eta_min())
    r = cs.r
    pi = sol.y[qp.dims["rs"]["bal"]]
    np.testing.assert_allclose(pi, [cA + r * (DA + F), cB + r * (DB - F)], rtol=1e-10)
    pay = D.planner_objective(qp, sol.x, 0.0, sol.y, 1.0) - D.planner_objective(qp, sol.x, 0.0)
    np.testing.assert_allclose(pay, DA * pi[0] + DB * pi[1], rtol=1e-12)
    g0 = Gm.scenario_gradient(qp, sol, 0.0)["grad"]
    g1 = Gm.scenario_gradient(qp, sol, 0.0, lmp=1.0)["grad"]
    np.testing.assert_allclose(g1 - g0, [0.0, 0.0, r * (DA - DB)], atol=1e-9)


def test_payments_jump_with_the_marginal_unit():
    # a generator's capacity decides which unit is marginal: below the load,
    # the expensive unit sets the price; the payments' derivative through a
    # held capacity is -r times the load-weighted price sensitivity
    cs = cases.single_node([30.0, 45.0], [80.0, 100.0], 120.0)
    qp, sol = D.solve_scenario(cs, 0, cs.eta_min())
    # unit 0 at its capacity 80, unit 1 marginal at 40: pi = 45 + 40 r;
    # one more MW of unit 0 takes one MW off unit 1: d pi / d eta_0 = -r
    r = cs.r
    np.testing.assert_allclose(sol.y[0], 45.0 + 40.0 * r, rtol=1e-10)
    g1 = Gm.scenario_gradient(qp, sol, 0.0, lmp=1.0)["grad"] - Gm.scenario_gradient(qp, sol, 0.0)["grad"]
    np.testing.assert_allclose(g1, [-r * 120.0, 0.0], atol=1e-9)


@pytest.mark.parametrize("lmp", [1.0, 0.3])
def test_payments_gradient_matches_resolves(lmp):
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=1, seed=7)
    eta = cases.jitter(cs.eta_min(), 3, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    qp, sol = D.solve_scenario(cs, 0, eta)
    gr = Gm.scenario_gradient(qp, sol, 50.0, lmp=lmp)["grad"]
    fd = Gm.fixed_set_differences(qp, sol, 50.0, lmp=lmp)
    ok = fd["ok"]
    scale = np.abs(gr).max()
    assert np.abs(fd["central"][ok] - gr[ok]).max() <= 1e-6 * scale
    # full re-solves on the coordinates with the largest price effect
    g0 = Gm.scenario_gradient(qp, sol, 50.0)["grad"]
    js = [int(j) for j in np.argsort(-np.abs(gr - g0)) if ok[j]][:6]
    h = 1e-3
    for j in js:
        vals = []
        for sgn in (1, -1):
            e2 = eta.copy()
            e2[j] += sgn * h
            q2, s2 = D.solve_scenario(cs, 0, e2)
            vals.append(D.planner_objective(q2, s2.x, 50.0, s2.y, lmp))
        np.testing.assert_allclose((vals[0] - vals[1]) / (2 * h), gr[j], atol=1e-5 * scale)
