"""GPU parity: the HIP dispatch solve and capacity gradient (through the
C-ABI) against the FP64 oracle.

Bars (from the planning problem's tolerances): relative objective gap
<= 1e-4 per scenario, relative KKT residual <= 1e-4 recomputed by the oracle
from the GPU's (x, y), gradient relative error (2-norm) <= 1e-3 at capacities
jittered off kinks."""
import numpy as np
import pytest

from paper_2410_13055_amd import cases
from oracle import dispatch as D
from oracle import gradient as Gm

pytestmark = pytest.mark.gpu

TOL = 1e-4
# the GPU stops at a KKT residual of 1e-4 computed from its FP32 iterate; the
# oracle recomputes it in FP64 from the same FP32 values with FP64 bounds
KKT_SLACK = 1.05


def _plan(case, **kw):
    from paper_2410_13055_amd import gridplan as gpb
    print(f"\n[gpu] plan {case.name} S={len(case.scenarios)} opts={kw}", flush=True)
    return gpb.Plan(case, gpb.options(**kw), stream=gpb.current_stream())


def _eta(case, seed=1):
    return cases.jitter(case.eta_min(), seed, eta_min=case.eta_min(), eta_max=case.eta_max())


def _oracle(case, s, eta, omega=0.0):
    off = case.eta_offsets()
    net = case.scenarios[s].network
    qp = D.assemble(case, s, eta[off[net]:off[net + 1]])
    sol = D.solve(qp)
    gr = Gm.scenario_gradient(qp, sol, omega)
    return qp, sol, gr


def _check_scenario(case, plan, s, eta, cost, stats, omega=0.0, check_grad=True):
    qp, sol, gr = _oracle(case, s, eta, omega)
    x, y = plan.solution(s)
    assert stats["status"] == 0, stats
    assert stats["kkt"] <= TOL
    res = D.kkt_residual(qp, x.astype(np.float64), y)
    assert res["kkt"] <= KKT_SLACK * TOL, res
    gap = abs(cost - sol.obj) / max(1.0, abs(sol.obj))
    assert gap <= TOL, (cost, sol.obj, gap)
    # the GPU's FP64 objective equals the oracle's evaluation of its x
    assert abs(cost - D.primal_objective(qp, x.astype(np.float64))) <= 1e-9 * abs(cost) + 1e-6
    return qp, sol, gr


def test_tiny_case_objective_and_certificate():
    cs = cases.config0()
    eta = _eta(cs)
    with _plan(cs) as p:
        cost, st, rc = p.solve(eta, [0])
        assert rc == 0
        _check_scenario(cs, p, 0, eta, cost[0], st[0])


@pytest.mark.parametrize("omega", [0.0, 50.0])
def test_tiny_case_gradient(omega):
    cs = cases.config0()
    eta = _eta(cs, 2)
    with _plan(cs) as p:
        cost, st, rc = p.solve(eta, [0])
        g, h, rc2 = p.grad([0], omega)
        assert rc2 == 0
    qp, sol, gr = _oracle(cs, 0, eta, omega)
    ref = cs.scenarios[0].weight * gr["grad"]
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    assert err <= 1e-3, (err, g, ref)
    href = cs.scenarios[0].weight * D.planner_objective(qp, sol.x, omega)
    assert abs(h - href) <= TOL * abs(href)


def test_two_node_closed_form():
    cA, cB, PA, PB, Dm, F, beta = 20.0, 60.0, 300.0, 200.0, 150.0, 80.0, 10.0
    cs = cases.two_node(cA, cB, PA, PB, Dm, F, beta)
    # prices are not bounded by a 1e-4 KKT residual; solve this closed form
    # to a tighter residual so that they are
    with _plan(cs, tol=1e-7) as p:
        cost, st, rc = p.solve(cs.eta_min(), [0])
        x, y = p.solution(0)
        g, _, _ = p.grad([0])
    # x = [pA, pB | f | thA, thB | uA, uB]
    np.testing.assert_allclose(x[[0, 1, 2]], [F, Dm - F, F], rtol=2e-3, atol=0.05)
    r = cs.r
    np.testing.assert_allclose(y[:2], [cA + r * F, cB + r * (Dm - F)], rtol=1e-3)
    dVdF = -(cB - cA) + r * (3 * F - Dm + F / (2 * beta ** 2))
    w = cs.scenarios[0].weight
    assert abs(g[2] - w * dVdF) <= 1e-3 * abs(w * dVdF)
    assert abs(g[0]) <= 1e-3 * abs(w * dVdF) and abs(g[1]) <= 1e-3 * abs(w * dVdF)


@pytest.mark.parametrize("Dm", [95.0, 400.0])
def test_single_node_no_lines_no_batteries(Dm):
    cs = cases.single_node([30.0, 45.0, 60.0, 75.0], [50.0, 80.0, 60.0, 70.0], Dm)
    with _plan(cs) as p:
        cost, st, rc = p.solve(cs.eta_min(), [0])
        _check_scenario(cs, p, 0, cs.eta_min(), cost[0], st[0])


def test_small_network_batch_several_tiles():
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=3, seed=7)
    eta = _eta(cs, 4)
    with _plan(cs) as p:
        cost, st, rc = p.solve(eta, [0, 1, 2])
        assert rc == 0
        for s in range(3):
            _check_scenario(cs, p, s, eta, cost[s], st[s])
        g, h, _ = p.grad([0, 1, 2])
    ref = np.zeros(cs.K)
    for s in range(3):
        _, _, gr = _oracle(cs, s, eta)
        ref += cs.scenarios[s].weight * gr["grad"] / 3
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) <= 1e-3


def test_emissions_gradient_small_network():
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=1, seed=9, omega=50.0)
    eta = _eta(cs, 5)
    with _plan(cs) as p:
        p.solve(eta, [0])
        g, h, rc = p.grad([0], 50.0)
    _, _, gr = _oracle(cs, 0, eta, 50.0)
    ref = cs.scenarios[0].weight * gr["grad"]
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) <= 1e-3


def test_batch_composition_does_not_change_results():
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=3, seed=7)
    eta = _eta(cs, 4)
    with _plan(cs, block=256, variant=1, check_every=64) as p:
        p.solve(eta, [0, 1, 2])
        xa, ya = p.solution(1)
        p.solve(eta, [1])
        xb, yb = p.solution(1)
        p.solve(eta, [2, 1])
        xc, yc = p.solution(1)
    np.testing.assert_array_equal(xa, xb)
    np.testing.assert_array_equal(ya, yb)
    np.testing.assert_array_equal(xa, xc)


def test_graph_replay_equals_eager():
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=2, seed=7)
    eta = _eta(cs, 4)
    fixed = dict(block=256, variant=1, check_every=64)   # no tuner: same launches
    with _plan(cs, **fixed) as p:
        p.solve(eta, [0, 1])
        xg, yg = p.solution(0)
    with _plan(cs, no_graph=1, **fixed) as p:
        p.solve(eta, [0, 1])
        xe, ye = p.solution(0)
    np.testing.assert_array_equal(xg, xe)
    np.testing.assert_array_equal(yg, ye)


@pytest.mark.parametrize("block", [64, 128, 512])
def test_block_size_does_not_change_results(block):
    cs = cases.config0()
    eta = _eta(cs)
    with _plan(cs, block=block) as p:
        cost, st, rc = p.solve(eta, [0])
        _check_scenario(cs, p, 0, eta, cost[0], st[0])


def test_warm_start_reaches_same_point_faster():
    cs = cases.config0()
    eta = _eta(cs)
    with _plan(cs) as p:
        c0, s0, _ = p.solve(eta, [0])
        eta2 = np.minimum(eta * 1.01, cs.eta_max())
        c1, s1, _ = p.solve(eta2, [0], warm=1)
        c2, s2, _ = p.solve(eta2, [0], warm=0)
    assert abs(c1[0] - c2[0]) <= 2 * TOL * abs(c2[0])
    assert s1[0]["iters"] <= s2[0]["iters"]


def test_plan_step_is_projected_gradient_step():
    cs = cases.config0()
    eta = cs.eta_min().copy()
    gamma = cs.gamma()
    alpha = 1e-4
    with _plan(cs) as p:
        eta_new, phi, delta, rc = p.step(alpha, [0], gamma, eta, omega=0.0, warm=0)
        p.solve(eta, [0])
        g, h, _ = p.grad([0])
    np.testing.assert_allclose(delta, gamma + g, rtol=1e-3, atol=1e-3 * np.abs(g).max())
    np.testing.assert_allclose(eta_new, np.clip(eta - alpha * delta, cs.eta_min(), cs.eta_max()), rtol=1e-12)
    assert abs(phi - (gamma @ eta + h)) <= TOL * abs(phi)


def test_full_size_certificate_on_two_scenarios():
    """At the 240-node, 168-hour size the oracle certifies the GPU's pair
    from its KKT residual and exact dual function (no full re-solve)."""
    cs = cases.config1(S=2)
    eta = cs.eta_min()
    with _plan(cs) as p:
        cost, st, rc = p.solve(eta, [0, 1])
        assert rc == 0
        for s in range(2):
            x, y = p.solution(s)
            qp = D.assemble(cs, s, eta)
            res = D.kkt_residual(qp, x.astype(np.float64), y)
            assert res["kkt"] <= KKT_SLACK * TOL, res
            # weak duality bounds the objective gap by the certified gap
            assert (res["P"] - res["D"]) <= TOL * (1 + abs(res["P"]))
            assert abs(cost[s] - res["P"]) <= 1e-9 * abs(cost[s])


@pytest.mark.parametrize("cfg", [3, 4])
def test_larger_workloads_certified_by_the_oracle(cfg):
    """500- and 1000-node workloads (T = 168) in the tuned launch
    configuration the benchmark uses: the oracle assembles each problem on
    its own and certifies the GPU's pair by its KKT residual and exact dual
    function (a full oracle re-solve at this size takes hours)."""
    cs = cases.by_id(cfg)
    eta = cs.eta_min()
    with _plan(cs) as p:
        cost, st, rc = p.solve(eta, [0, 1])
        assert rc == 0
        sols = [p.solution(s) for s in (0, 1)]
    for s, (x, y) in enumerate(sols):
        qp = D.assemble(cs, s, eta)
        res = D.kkt_residual(qp, x.astype(np.float64), y)
        print(f"\n[gpu] config {cfg} scenario {s}: oracle KKT {res['kkt']:.2e}", flush=True)
        assert res["kkt"] <= KKT_SLACK * TOL, res
        assert (res["P"] - res["D"]) <= TOL * (1 + abs(res["P"]))
        assert abs(cost[s] - res["P"]) <= 1e-9 * abs(cost[s])


def test_emissions_gradient_where_the_adjoint_is_nearly_zero():
    """100-node case at 200 $/t: most gas units sit at a bound, so the adjoint
    solution is small and its objective near zero; the adjoint solve must
    still stop (its gap is measured against the dual function at zero) and
    match the oracle gradient over the coordinates at which the map is
    differentiable (fixed-active-set verification at +-1e-3 MW)."""
    cs = cases.geo100()
    s, omega = 1, 200.0
    eta = _eta(cs, 5)
    with _plan(cs) as p:
        p.solve(eta, [s])
        g, h, rc = p.grad([s], omega)
    assert rc == 0
    qp, sol, gr = _oracle(cs, s, eta, omega)
    w = cs.scenarios[s].weight
    ref = w * gr["grad"]
    ok = Gm.fixed_set_differences(qp, sol, omega, h=1e-3)["ok"]
    err = np.linalg.norm((g - ref)[ok]) / np.linalg.norm(ref[ok])
    print(f"\n[gpu] geo100 emissions gradient err {err:.2e} over {int(ok.sum())} of {ok.size} coordinates",
          flush=True)
    assert err <= 1e-3


@pytest.mark.parametrize("PA,PB,F,cA,cB", [(300.0, 200.0, 0.0, 20.0, 60.0), (300.0, 200.0, 0.0, 60.0, 20.0),
                                          (300.0, 0.0, 80.0, 20.0, 60.0)])
def test_zero_capacity_one_sided_gradient(PA, PB, F, cA, cB):
    """A line or a generator at zero capacity: the GPU returns the derivative
    for increasing capacity, -|z_f| for the line and -(pi_B - c_B) for the
    generator, as the oracle does (whose value the closed forms pin)."""
    cs = cases.two_loads(PA, PB, F, cA=cA, cB=cB)
    eta = cs.eta_min()
    with _plan(cs) as p:
        cost, st, rc = p.solve(eta, [0])
        assert rc == 0, st
        g, _, _ = p.grad([0], 0.0, eta=eta)
    qp, sol, gr = _oracle(cs, 0, eta)
    ref = cs.scenarios[0].weight * gr["grad"]
    print(f"\n[gpu] zero capacity: gpu {g} oracle {ref}", flush=True)
    assert np.linalg.norm(g - ref) <= 1e-3 * np.linalg.norm(ref)
    assert np.all(g <= 0.0)
