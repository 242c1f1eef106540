"""Pins of the oracle's certificate and gradient pieces on points that are
not the optimum, with values worked by hand from the definitions:

- the relative KKT residual triple (the solver-independent stopping test of
  the dispatch map, eq. (2)) on pairs moved off the optimum by a known amount;
- the one-sided capacity derivative at zero capacity (Section 2.2's gradient
  at the edge of the box), from the two-node optimality conditions;
- the fixed-active-set central differences against full re-solves;
- every column of the warm-start features on a hand-built network.
"""
import numpy as np
import pytest

from paper_2410_13055_amd import cases
from oracle import dispatch as D
from oracle import gradient as Gm
from oracle import mlp as M


def _two_node_solved():
    cs = cases.two_node(20.0, 60.0, 300.0, 200.0, 150.0, 80.0, 10.0)
    qp, sol = D.solve_scenario(cs, 0, cs.eta_min())
    assert sol.polished
    return cs, qp, sol


def test_primal_residual_of_a_moved_generator():
    """Moving p_B by delta leaves only node B's balance row off by delta:
    r_pri = delta / (1 + ||e||_inf), ||e||_inf = the load 150 MW."""
    _, qp, sol = _two_node_solved()
    vs = qp.dims["vs"]
    for delta in (0.5, 3.0):
        x = sol.x.copy()
        x[vs["p"].start + 1] += delta
        res = D.kkt_residual(qp, x, sol.y)
        assert res["r_pri"] == pytest.approx(delta / (1.0 + 150.0), rel=1e-9)


def test_dual_residual_counts_the_angles_only():
    """Moving the flow dual mu by dm changes E'y on the two angles by -+beta dm
    and on the (boxed) flow by dm.  Only the angles are free, so
    r_dual = beta |dm| / (1 + ||q||_inf), ||q||_inf = lambda_u = 1e4; the
    congested flow's multiplier (about 40 $/MWh) must not enter."""
    cs, qp, sol = _two_node_solved()
    beta = float(cs.networks[0].line_beta[0])
    rs = qp.dims["rs"]
    for dm in (0.25, -2.0):
        y = sol.y.copy()
        y[rs["flow"].start] += dm
        res = D.kkt_residual(qp, sol.x, y)
        assert res["r_dual"] == pytest.approx(beta * abs(dm) / (1.0 + 1e4), rel=1e-6)


def test_gap_of_a_single_node_pair_worked_by_hand():
    """One node, one generator (c = 20 $/MWh, cap 100 MW), load 50 MW, T = 1.
    x = (p = 50, th = 0, u = 0), y = pi = 20.03:
      P = 20*50 + (r/2) 50^2 = 1001.25
      D = min_{0<=p<=100} (20 - 20.03) p + (r/2) p^2   (p = 30: -0.45)
          + min_{u>=0} (1e4 - 20.03) u + (r/2) u^2       (u = 0: 0)
          + min_th (r/2) th^2                            (0)
          + 50 * 20.03                                   (1001.5)
        = 1001.05
      r_gap = 0.2 / (1 + 1001.25).
    An infeasible x (p = 40) has P = 800 + 0.8 = 800.8 below D, and the gap is
    measured against the larger of the two: r_gap = 200.25 / (1 + 1001.05)."""
    cs = cases.single_node([20.0], [100.0], 50.0)
    qp = D.assemble(cs, 0, cs.eta_min())
    vs = qp.dims["vs"]
    x = np.zeros(qp.n)
    x[vs["p"]] = 50.0
    y = np.array([20.03])
    res = D.kkt_residual(qp, x, y)
    assert res["P"] == pytest.approx(1001.25, rel=1e-12)
    assert res["D"] == pytest.approx(1001.05, rel=1e-9)
    assert res["r_gap"] == pytest.approx(0.2 / 1002.25, rel=1e-6)
    assert res["r_pri"] == pytest.approx(0.0, abs=1e-15)
    x[vs["p"]] = 40.0
    res = D.kkt_residual(qp, x, y)
    assert res["P"] == pytest.approx(800.8, rel=1e-12)
    assert res["r_gap"] == pytest.approx(200.25 / 1002.05, rel=1e-6)


def test_box_violation():
    """p_B set 2 MW above its 200 MW cap: r_box = 2 / (1 + 300), 300 MW being
    the largest finite bound (generator A's cap)."""
    _, qp, sol = _two_node_solved()
    vs = qp.dims["vs"]
    x = sol.x.copy()
    x[vs["p"].start + 1] = 202.0
    res = D.kkt_residual(qp, x, sol.y)
    assert res["r_box"] == pytest.approx(2.0 / 301.0, rel=1e-9)
    assert res["kkt"] >= res["r_box"]


# --------------------------------------------------------------------------
# zero capacity: the derivative for increasing capacity
# --------------------------------------------------------------------------

def _two_loads(PA, PB, F, **kw):
    return cases.two_loads(PA, PB, F, **kw)


def test_zero_line_capacity_one_sided_derivative():
    """F = 0: the nodes clear alone, pi_A = cA + r DA, pi_B = cB + r DB, and
    the angles and mu are zero, so the flow multiplier is
    z_f = pi_B - pi_A = (cB - cA) + r (DB - DA) > 0; opening the line by dF
    saves z_f dF: d+V/dF = -z_f.  Forward differences of full re-solves
    agree."""
    cs = _two_loads(300.0, 200.0, 0.0)
    eta = cs.eta_min()
    qp, sol = D.solve_scenario(cs, 0, eta)
    r = cs.r
    zf = (60.0 - 20.0) + r * (150.0 - 50.0)
    g = Gm.scenario_gradient(qp, sol, 0.0)["grad"]
    assert g[2] == pytest.approx(-zf, rel=1e-9)
    assert g[0] == pytest.approx(0.0, abs=1e-9) and g[1] == pytest.approx(0.0, abs=1e-9)
    h = 1e-3
    ep = eta.copy()
    ep[2] += h
    fwd = (Gm.value(cs, 0, ep, 0.0) - Gm.value(cs, 0, eta, 0.0)) / h
    assert fwd == pytest.approx(-zf, rel=1e-4)


def test_zero_line_capacity_reversed_flow_direction():
    """With the cheap unit at the line's 'to' end the flow would run against
    the line's orientation: z_f = pi_B - pi_A < 0 and d+V/dF = -|z_f|."""
    cs = _two_loads(300.0, 200.0, 0.0, cA=60.0, cB=20.0)
    qp, sol = D.solve_scenario(cs, 0, cs.eta_min())
    zf = (20.0 - 60.0) + cs.r * (150.0 - 50.0)
    g = Gm.scenario_gradient(qp, sol, 0.0)["grad"]
    assert g[2] == pytest.approx(-abs(zf), rel=1e-9)


def test_zero_generator_capacity_one_sided_derivative():
    """Generator B at zero capacity: node B imports F = 80 MW and sheds
    DB - F = 70 MW, so pi_B = lambda_u + r 70 and the generator's multiplier
    is z = pi_B - cB > 0: d+V/d eta_B = -(pi_B - cB).  Generator A at zero
    capacity with nothing to gain would have z <= 0 and derivative 0; here
    A is the marginal unit and keeps its capacity."""
    cs = _two_loads(300.0, 0.0, 80.0)
    eta = cs.eta_min()
    qp, sol = D.solve_scenario(cs, 0, eta)
    pib = cs.lambda_u + cs.r * 70.0
    g = Gm.scenario_gradient(qp, sol, 0.0)["grad"]
    assert g[1] == pytest.approx(-(pib - 60.0), rel=1e-9)
    h = 1e-3
    ep = eta.copy()
    ep[1] += h
    fwd = (Gm.value(cs, 0, ep, 0.0) - Gm.value(cs, 0, eta, 0.0)) / h
    assert fwd == pytest.approx(-(pib - 60.0), rel=1e-4)


def test_zero_generator_capacity_without_benefit_has_zero_derivative():
    """A second expensive unit at node A with zero capacity (cost 90 above
    pi_A): more capacity would not be used, d+V/d eta = 0."""
    base = _two_loads(300.0, 200.0, 80.0)
    net = base.networks[0]
    net.gen_node = np.array([0, 1, 0], np.int32)
    net.gen_kind = np.array([cases.GAS] * 3, np.int32)
    net.gen_cost = cases._f32([20.0, 60.0, 90.0])
    net.gen_emis = cases._f32([0.4] * 3)
    net.eta_min = cases._f32([300.0, 200.0, 0.0, 80.0])
    net.eta_max = cases._f32([700.0, 600.0, 400.0, 480.0])
    net.gamma = cases._f32([1e5] * 4)
    base.scenarios[0].avail = np.ones((3, 1))
    qp, sol = D.solve_scenario(base, 0, base.eta_min())
    g = Gm.scenario_gradient(qp, sol, 0.0)["grad"]
    assert g[2] == pytest.approx(0.0, abs=1e-9)


# --------------------------------------------------------------------------
# fixed-active-set differences
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mk,omega", [(cases.config0, 0.0), (cases.config0, 50.0),
                                      (lambda: cases.small_geo(n_nodes=10, G=24, B=2, T=8, S=1, seed=3), 50.0)])
def test_fixed_set_differences_match_gradient_and_full_resolves(mk, omega):
    """On every coordinate both of whose ends verify, the fixed-active-set
    central difference is the exact derivative of the quadratic piece: it
    equals the implicit gradient (to rounding) and the central difference of
    two full interior-point re-solves.  The re-solves' values carry a
    relative error of ~1e-11 (about 3e-4 $ on this 3e7 $ objective), so they
    are differenced at h = 0.05 MW, on coordinates whose ends verify at that
    step too."""
    cs = mk()
    eta = cases.jitter(cs.eta_min(), 5, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    qp = D.assemble(cs, 0, eta)
    sol = D.solve(qp)
    g = Gm.scenario_gradient(qp, sol, omega)["grad"]
    fd = Gm.fixed_set_differences(qp, sol, omega, h=1e-3)
    scale = np.abs(g).max()
    assert fd["ok"].sum() >= 0.8 * qp.K
    ok = fd["ok"]
    np.testing.assert_allclose(fd["central"][ok], g[ok], atol=1e-9 * scale)
    wide = Gm.fixed_set_differences(qp, sol, omega, h=0.05)
    np.testing.assert_allclose(wide["central"][wide["ok"]], g[wide["ok"]], atol=1e-9 * scale)
    both = np.where(ok & wide["ok"])[0]
    assert both.size >= 6
    for j in both[:: max(1, both.size // 6)]:
        full = Gm.central_difference(cs, 0, eta, int(j), omega, h=0.05)
        assert abs(full["central"] - fd["central"][j]) <= 1e-6 * scale, (j, full, fd["central"][j])


def test_fixed_set_differences_flag_a_kink():
    """Single node, two units, load exactly at the first unit's capacity:
    with more capacity the cheap unit takes it (its multiplier is positive:
    d+V/d eta_1 < 0), with less the dear unit fills in.  Moving eta_1 down by
    h releases the dear unit from its lower bound: the backward end fails to
    verify, so the coordinate is flagged, and the forward and backward
    full-resolve slopes differ."""
    cs = cases.single_node([20.0, 50.0], [100.0, 100.0], 100.0)
    eta = cs.eta_min()
    qp = D.assemble(cs, 0, eta)
    sol = D.solve(qp)
    fd = Gm.fixed_set_differences(qp, sol, 0.0, h=1e-3)
    assert not fd["ok"][0]
    full = Gm.central_difference(cs, 0, eta, 0, 0.0, h=1e-3)
    assert abs(full["forward"] - full["backward"]) > 1.0


# --------------------------------------------------------------------------
# warm-start features, every column
# --------------------------------------------------------------------------

def test_feature_columns_on_a_hand_built_network():
    """Node 0: gas unit (300 MW), loads 10/20 MW.  Node 1: solar unit
    (100 MW, availability 0.5/0.25), battery 25 MW, loads 150/160 MW.  Line
    0 -> 1 of 80 MW.  Columns (MW/100): own load, renewable available, thermal
    available, neighbours' load, neighbours' renewable available (T each),
    then battery, incident line and thermal nameplate capacity."""
    net = cases.Network(
        n_nodes=2, line_from=np.array([0], np.int32), line_to=np.array([1], np.int32),
        line_beta=cases._f32([10.0]), gen_node=np.array([0, 1], np.int32),
        gen_kind=np.array([cases.GAS, cases.SOLAR], np.int32), gen_cost=cases._f32([20.0, 0.0]),
        gen_emis=cases._f32([0.4, 0.0]), batt_node=np.array([1], np.int32),
        eta_min=cases._f32([300.0, 100.0, 80.0, 25.0]), eta_max=cases._f32([600.0, 200.0, 160.0, 50.0]),
        gamma=cases._f32([1e5] * 4))
    sc = cases.Scenario(network=0, T=2, avail=np.array([[1.0, 1.0], [0.5, 0.25]]),
                        load=cases._f32([[10.0, 20.0], [150.0, 160.0]]), weight=4380.0)
    cs = cases.Case(name="feat", networks=[net], scenarios=[sc])
    X = M.features(cs, 0, cs.eta_min()) * 100.0
    want = np.array([
        [10, 20, 0, 0, 300, 300, 150, 160, 50, 25, 0, 80, 300],
        [150, 160, 50, 25, 0, 0, 10, 20, 0, 0, 25, 80, 0],
    ], dtype=float)
    np.testing.assert_allclose(X, want, rtol=1e-12, atol=1e-12)


def test_neighbour_and_capacity_columns_on_the_ring():
    """Ring of 6 plus chords (0,3), (2,5): degrees 3,2,3,3,2,3.  Summed over
    nodes, the neighbours' load column counts every node's load once per
    incident line, the incident line capacity counts every line twice, and
    the battery and thermal columns sum to the fleets' capacities."""
    cs = cases.config0()
    eta = cases.jitter(cs.eta_min(), 2, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    net, sc = cs.networks[0], cs.scenarios[0]
    T, G, L = sc.T, net.n_gens, net.n_lines
    X = M.features(cs, 0, eta) * 100.0
    deg = np.array([3, 2, 3, 3, 2, 3], float)
    np.testing.assert_allclose(X[:, 3 * T:4 * T].sum(0), (deg[:, None] * sc.load).sum(0), rtol=1e-12)
    ren = np.where(net.gen_cost == 0)[0]
    ren_at = np.zeros((net.n_nodes, T))
    for g in ren:
        ren_at[net.gen_node[g]] += sc.avail[g] * eta[g]
    np.testing.assert_allclose(X[:, 4 * T:5 * T].sum(0), (deg[:, None] * ren_at).sum(0), rtol=1e-12)
    np.testing.assert_allclose(X[:, 5 * T].sum(), eta[G + L:].sum(), rtol=1e-12)
    np.testing.assert_allclose(X[:, 5 * T + 1].sum(), 2 * eta[G:G + L].sum(), rtol=1e-12)
    np.testing.assert_allclose(X[:, 5 * T + 2].sum(), eta[:G][net.gen_cost > 0].sum(), rtol=1e-12)


def test_kink_distance_on_the_two_node_closed_form():
    """Two-node congested case (cA 20, cB 60, load 150 at B, line 80 MW):
    raising the line capacity moves flow onto it one for one and takes B's
    output down, which reaches zero at F = 150, 70 MW away; lowering it keeps
    every classification until the box collapses at zero.  The nearest kink
    along F is therefore 70 MW away, and the curvature of V along F is
    r (|df|^2 + |dp_A|^2 + |dp_B|^2 + |dth|^2) = r (3 + 1 / (2 beta^2)).
    The generators run below their capacities (A at 80 of 300 MW, B at 70 of
    200 MW): lowering a capacity meets the output 220 and 130 MW away, and
    along them V is flat."""
    cs = cases.two_node(20.0, 60.0, 300.0, 200.0, 150.0, 80.0, 10.0)
    qp, sol = D.solve_scenario(cs, 0, cs.eta_min())
    fd = Gm.fixed_set_differences(qp, sol, 0.0, h=1e-3)
    assert fd["dist"][2] == pytest.approx(70.0, rel=1e-9)
    assert fd["dist"][0] == pytest.approx(220.0, rel=1e-9)
    assert fd["dist"][1] == pytest.approx(130.0, rel=1e-9)
    assert fd["curv"][0] == 0.0 and fd["curv"][1] == 0.0
    beta = float(cs.networks[0].line_beta[0])
    assert fd["curv"][2] == pytest.approx(cs.r * (3.0 + 1.0 / (2 * beta ** 2)), rel=1e-9)
