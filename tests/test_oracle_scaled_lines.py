"""Pins for a constraint matrix that depends on the capacities (Section 2.1
writes the dispatch constraints as A_s(eta) x <= b_s(eta)): an AC line's
susceptance scales with its capacity, beta_l(eta) = beta_l * eta_l /
eta_min_l, as for an expanded corridor of parallel circuits.

The capacity derivative then gains the terms of dE (the implicit function
theorem with a moving matrix); the closed form below and full re-solves pin
them."""
import numpy as np
import pytest

from paper_2410_13055_amd import cases
from oracle import dispatch as D
from oracle import gradient as Gm


def _solve(case, eta=None, s=0):
    eta = case.eta_min() if eta is None else eta
    return D.solve_scenario(case, s, eta)


@pytest.mark.parametrize("F", [80.0, 120.0])
def test_scaled_two_node_closed_form(F):
    # the line is full (p_A = f = F, p_B = D - F) and its angles split the
    # difference: th_A = -th_B = F / (2 beta(F)) with beta(F) = beta F / F0,
    # so the angle regulariser r/2 (th_A^2 + th_B^2) = r F0^2 / (4 beta^2) no
    # longer depends on F, and dV/dF = cA - cB + r (3F - D) (the fixed-beta
    # line adds r F / (2 beta^2))
    cA, cB, D_, F0, beta = 20.0, 60.0, 250.0, 80.0, 10.0
    cs = cases.scaled_two_node(cA=cA, cB=cB, D=D_, F=F0, beta=beta)
    eta = cs.eta_min().copy()
    eta[2] = F
    qp, sol = _solve(cs, eta)
    r = cs.r
    vs = qp.dims["vs"]
    bF = beta * F / F0
    np.testing.assert_allclose(qp.E.toarray()[2, vs["th"]], [-bF, bF], rtol=1e-15)
    x = sol.x
    np.testing.assert_allclose(x[vs["p"]], [F, D_ - F], atol=1e-7)
    np.testing.assert_allclose(x[vs["th"]], [F / (2 * bF), -F / (2 * bF)], atol=1e-9)
    V = cA * F + cB * (D_ - F) + 0.5 * r * (2 * F ** 2 + (D_ - F) ** 2 + F0 ** 2 / (2 * beta ** 2))
    assert abs(sol.obj - V) <= 1e-9 * V
    gr = Gm.scenario_gradient(qp, sol, 0.0)
    np.testing.assert_allclose(gr["grad"], [0.0, 0.0, cA - cB + r * (3 * F - D_)], atol=1e-7)
    np.testing.assert_allclose(gr["envelope"], gr["grad"], atol=1e-9)
    # the same line with a fixed susceptance
    fx = cases.two_node(cA=cA, cB=cB, D=D_, F=F0, beta=bF)
    fx.networks[0].eta_min[2] = F
    qf, sf = _solve(fx, eta)
    gf = Gm.scenario_gradient(qf, sf, 0.0)["grad"][2]
    np.testing.assert_allclose(gf - gr["grad"][2], r * F / (2 * bF ** 2), rtol=1e-6)


@pytest.mark.parametrize("omega", [0.0, 200.0])
def test_scaled_network_gradient_matches_resolves(omega):
    # every line capacity and a few others: central differences of full
    # re-solves (h = 0.05 MW) against the adjoint gradient with the dE terms
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=1, seed=7, beta_scales=True)
    net = cs.networks[0]
    eta = cases.jitter(cs.eta_min(), 3, amount=5.0, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    qp, sol = _solve(cs, eta)
    gr = Gm.scenario_gradient(qp, sol, omega)["grad"]
    scale = np.abs(gr).max()
    G, L = net.n_gens, net.n_lines
    js = list(range(G, G + L)) + [0, 5, G + L]
    h = 0.05
    bad = []
    for j in js:
        vals = []
        for sgn in (1, -1):
            e2 = eta.copy()
            e2[j] += sgn * h
            q2, s2 = _solve(cs, e2)
            vals.append(D.planner_objective(q2, s2.x, omega))
        fd = (vals[0] - vals[1]) / (2 * h)
        if abs(fd - gr[j]) > 1e-5 * scale:
            bad.append((j, fd, gr[j]))
    assert not bad, bad


def test_matrix_terms_vanish_without_scaling():
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=1, seed=7)
    qp, sol = _solve(cs)
    assert qp.line_dbeta is None
    sc = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=1, seed=7, beta_scales=True)
    qs, ss = _solve(sc)
    # at eta_min both networks are the same, so are the solutions; only the
    # line derivatives differ, by the dE terms
    np.testing.assert_allclose(ss.x, sol.x, atol=1e-9)
    g0 = Gm.scenario_gradient(qp, sol, 0.0)["grad"]
    g1 = Gm.scenario_gradient(qs, ss, 0.0)["grad"]
    net = cs.networks[0]
    G, L = net.n_gens, net.n_lines
    np.testing.assert_allclose(g1[:G], g0[:G], atol=1e-9)
    np.testing.assert_allclose(g1[G + L:], g0[G + L:], atol=1e-9)
    assert np.abs(g1[G:G + L] - g0[G:G + L]).max() > 1e-3
