"""GPU parity for a constraint matrix that depends on the capacities
(Section 2.1's A_s(eta)): AC susceptances that scale with line capacity,
beta_l(eta) = line_beta_l * eta_l / eta_min_l.  The library recomputes the
susceptances and the angle weights from eta at every solve and adds the
matrix terms to the gradient (forward pass and adjoint pass); the oracle's
values are pinned by a closed form and full re-solves.

Bars as in the other dispatch tests: KKT residual <= 1e-4 recomputed by the
oracle from the GPU's (x, y), objective gap <= 1e-4, gradient relative error
<= 1e-3."""
import numpy as np
import pytest

from paper_2410_13055_amd import cases
from oracle import dispatch as D
from oracle import gradient as Gm

pytestmark = pytest.mark.gpu

TOL = 1e-4
KKT_SLACK = 1.05


def _plan(case, **kw):
    from paper_2410_13055_amd import gridplan as gpb
    print(f"\n[gpu] plan {case.name} S={len(case.scenarios)} opts={kw}", flush=True)
    return gpb.Plan(case, gpb.options(**kw), stream=gpb.current_stream())


def test_scaled_two_node_closed_form():
    cA, cB, D_, F0, beta, F = 20.0, 60.0, 250.0, 80.0, 10.0, 120.0
    cs = cases.scaled_two_node(cA=cA, cB=cB, D=D_, F=F0, beta=beta)
    eta = cs.eta_min().copy()
    eta[2] = F
    with _plan(cs, tol=1e-7) as p:
        cost, st, rc = p.solve(eta, [0])
        assert rc == 0, st
        x, y = p.solution(0)
        g, _, _ = p.grad([0], 0.0, eta=eta)
    bF = beta * F / F0
    # x = [pA, pB | f | thA, thB | uA, uB]
    np.testing.assert_allclose(x[[0, 1, 2]], [F, D_ - F, F], rtol=2e-3, atol=0.05)
    np.testing.assert_allclose(x[[3, 4]], [F / (2 * bF), -F / (2 * bF)], rtol=2e-3)
    w = cs.scenarios[0].weight
    ref = w * (cA - cB + cs.r * (3 * F - D_))
    assert abs(g[2] - ref) <= 1e-3 * abs(ref)


@pytest.mark.parametrize("T", [24, 22])
@pytest.mark.parametrize("omega", [0.0, 200.0])
def test_scaled_network_against_oracle(T, omega):
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=T, S=2, seed=7, beta_scales=True)
    net = cs.networks[0]
    lo, hi = cs.eta_min(), cs.eta_max()
    etas = [cases.jitter(lo, 3, amount=5.0, eta_min=lo, eta_max=hi),
            cases.jitter(lo, 4, amount=40.0, eta_min=lo, eta_max=hi)]
    G, L = net.n_gens, net.n_lines
    with _plan(cs) as p:
        for k, eta in enumerate(etas):   # the second solve moves every susceptance
            cost, st, rc = p.solve(eta, [0, 1])
            assert rc == 0, st
            sols = [p.solution(s) for s in (0, 1)]
            g, h, rc2 = p.grad([0, 1], omega, eta=eta)
            assert rc2 == 0
            ref = np.zeros(cs.K)
            href = 0.0
            for s in (0, 1):
                qp = D.assemble(cs, s, eta)
                sol = D.solve(qp)
                x, y = sols[s]
                res = D.kkt_residual(qp, x.astype(np.float64), y)
                assert res["kkt"] <= KKT_SLACK * TOL, res
                assert abs(cost[s] - sol.obj) <= TOL * abs(sol.obj)
                ref += cs.scenarios[s].weight * Gm.scenario_gradient(qp, sol, omega)["grad"] / 2
                href += cs.scenarios[s].weight * D.planner_objective(qp, sol.x, omega) / 2
            err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
            el = np.linalg.norm((g - ref)[G:G + L]) / np.linalg.norm(ref[G:G + L])
            print(f"[gpu] scaled lines T={T} omega={omega} eta {k}: gradient err {err:.2e}, lines {el:.2e}",
                  flush=True)
            assert err <= 1e-3
            assert el <= 1e-3
            assert abs(h - href) <= TOL * abs(href)
