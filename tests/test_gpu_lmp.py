"""GPU parity for a planner objective on the prices: h_s = c_s + omega *
emissions + lmp * sum pi D (Section 2.1 lets h_s depend on the LMPs).  The
library's adjoint solve carries lmp * load on its balance rows; the oracle
is pinned by closed forms and re-solves."""
import numpy as np
import pytest

from paper_2410_13055_amd import cases
from oracle import dispatch as D
from oracle import gradient as Gm

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _plan(case, **kw):
    from paper_2410_13055_amd import gridplan as gpb
    print(f"\n[gpu] plan {case.name} S={len(case.scenarios)} opts={kw}", flush=True)
    return gpb.Plan(case, gpb.options(**kw), stream=gpb.current_stream())


def test_two_load_payments_closed_form():
    cA, cB, DA, DB, F = 20.0, 60.0, 50.0, 150.0, 80.0
    cs = cases.two_loads(300.0, 200.0, F, DA=DA, DB=DB, cA=cA, cB=cB)
    eta = cs.eta_min()
    with _plan(cs, tol=1e-7) as p:
        p.solve(eta, [0])
        g0, h0, _ = p.grad([0], 0.0, eta=eta)
        p.set_price_weight(1.0)
        g1, h1, rc = p.grad([0], 0.0, eta=eta)
        assert rc == 0
        ho = p.objective([0], 0.0, eta=eta)
    w, r = cs.scenarios[0].weight, cs.r
    pay = DA * (cA + r * (DA + F)) + DB * (cB + r * (DB - F))
    assert abs((h1 - h0) - w * pay) <= 1e-6 * w * pay
    assert abs(ho - h1) <= 1e-9 * abs(h1)
    np.testing.assert_allclose(g1 - g0, [0.0, 0.0, w * r * (DA - DB)], atol=1e-3 * w * r * abs(DA - DB))


@pytest.mark.parametrize("T", [24, 22])
@pytest.mark.parametrize("omega", [0.0, 50.0])
def test_payments_gradient_against_oracle(T, omega):
    lmp = 0.5
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=T, S=2, seed=7)
    eta = cases.jitter(cs.eta_min(), 3, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    with _plan(cs) as p:
        p.set_price_weight(lmp)
        cost, st, rc = p.solve(eta, [0, 1])
        assert rc == 0, st
        g, h, rc2 = p.grad([0, 1], omega, eta=eta)
        assert rc2 == 0
    ref = np.zeros(cs.K)
    href = 0.0
    for s in (0, 1):
        qp = D.assemble(cs, s, eta)
        sol = D.solve(qp)
        ref += cs.scenarios[s].weight * Gm.scenario_gradient(qp, sol, omega, lmp=lmp)["grad"] / 2
        href += cs.scenarios[s].weight * D.planner_objective(qp, sol.x, omega, sol.y, lmp) / 2
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    print(f"[gpu] payments T={T} omega={omega}: gradient err {err:.2e}, h {h:.6e} (oracle {href:.6e})", flush=True)
    assert err <= 1e-3
    assert abs(h - href) <= TOL * abs(href)
