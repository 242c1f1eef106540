"""Pins for the FP64 oracle against facts that do not come from the oracle
itself: closed forms derived from the dispatch KKT conditions, the textbook
merit order, brute-force enumeration of active sets, duality certificates,
finite differences and invariants of the dispatch map (Section 2.1 eq. (2),
Section 2.2 gradient)."""
import itertools

import numpy as np
import pytest

from paper_2410_13055_amd import cases
from oracle import dispatch as D
from oracle import gradient as Gm


def _solve(case, eta=None, s=0):
    eta = case.eta_min() if eta is None else eta
    return D.solve_scenario(case, s, eta)


# --------------------------------------------------------------------------
# two-node congested line: closed form from the KKT conditions
# --------------------------------------------------------------------------

@pytest.mark.parametrize("cA,cB,PA,PB,Dm,F,beta", [
    (20.0, 60.0, 300.0, 200.0, 150.0, 80.0, 10.0),
    (35.0, 75.0, 500.0, 120.0, 210.0, 130.0, 6.0),
])
def test_two_node_congested_closed_form(cA, cB, PA, PB, Dm, F, beta):
    cs = cases.two_node(cA, cB, PA, PB, Dm, F, beta)
    qp, sol = _solve(cs)
    r = cs.r
    vs = qp.dims["vs"]
    x = sol.x
    assert sol.polished
    pA, pB = x[vs["p"]]
    f = x[vs["f"]][0]
    thA, thB = x[vs["th"]]
    np.testing.assert_allclose([pA, pB, f], [F, Dm - F, F], atol=1e-7)
    np.testing.assert_allclose([thA, thB], [F / (2 * beta), -F / (2 * beta)], atol=1e-9)
    np.testing.assert_allclose(x[vs["u"]], 0.0, atol=1e-7)
    pi = sol.y[qp.dims["rs"]["bal"]]
    np.testing.assert_allclose(pi, [cA + r * F, cB + r * (Dm - F)], rtol=1e-9)
    V = cA * F + cB * (Dm - F) + 0.5 * r * (2 * F ** 2 + (Dm - F) ** 2 + F ** 2 / (2 * beta ** 2))
    assert abs(sol.obj - V) <= 1e-9 * V
    dVdF = -(cB - cA) + r * (3 * F - Dm + F / (2 * beta ** 2))
    gr = Gm.scenario_gradient(qp, sol, 0.0)
    np.testing.assert_allclose(gr["grad"], [0.0, 0.0, dVdF], atol=1e-7)


def test_two_node_uncongested_single_price():
    cs = cases.two_node(20.0, 60.0, 300.0, 200.0, 50.0, 80.0, 10.0)
    qp, sol = _solve(cs)
    pi = sol.y[qp.dims["rs"]["bal"]]
    # with the line slack both nodes clear at the cheap unit's marginal price
    # up to the flow and angle regulariser terms
    assert abs(pi[0] - pi[1]) < 1e-1
    assert abs(pi[0] - (20.0 + cs.r * 50.0)) < 1e-1
    gr = Gm.scenario_gradient(qp, sol, 0.0)
    np.testing.assert_allclose(gr["grad"], 0.0, atol=1e-9)


# --------------------------------------------------------------------------
# single node: exact merit order by sorting breakpoints
# --------------------------------------------------------------------------

def _merit_order_price(costs, caps, Dm, r, lam):
    """Solve sum_g clip((pi-c_g)/r, 0, cap_g) + max(0, (pi-lam)/r) = D exactly:
    the left side is piecewise linear and increasing, so find the segment
    between sorted breakpoints and solve the linear equation there."""
    bps = sorted(set([c for c in costs] + [c + r * k for c, k in zip(costs, caps)] + [lam]))

    def S(pi):
        s = sum(min(max((pi - c) / r, 0.0), k) for c, k in zip(costs, caps))
        return s + max(0.0, (pi - lam) / r)

    lo = min(bps) - 1.0
    for b in bps + [lam + 1e9]:
        if S(b) >= Dm:
            hi = b
            break
        lo = b
    s_lo, s_hi = S(lo), S(hi)
    return lo + (Dm - s_lo) * (hi - lo) / (s_hi - s_lo)


@pytest.mark.parametrize("Dm", [10.0, 95.0, 150.0, 259.0, 400.0])
def test_single_node_merit_order(Dm):
    costs = [30.0, 45.0, 60.0, 75.0]
    caps = [50.0, 80.0, 60.0, 70.0]
    cs = cases.single_node(costs, caps, Dm)
    qp, sol = _solve(cs)
    pi = sol.y[qp.dims["rs"]["bal"]][0]
    ref = _merit_order_price(costs, caps, Dm, cs.r, cs.lambda_u)
    assert abs(pi - ref) <= 1e-7 * max(1.0, abs(ref))
    p = sol.x[qp.dims["vs"]["p"]]
    np.testing.assert_allclose(p, np.clip((ref - np.array(costs)) / cs.r, 0, caps), atol=1e-6)
    # as r -> 0 the price is the marginal unit's cost (textbook merit order)
    cum = np.cumsum(caps)
    if Dm < cum[-1]:
        marginal = costs[int(np.searchsorted(cum, Dm))]
        assert abs(pi - marginal) < 0.2
    else:
        assert pi >= cs.lambda_u - 1e-6  # shortage: scarcity price


# --------------------------------------------------------------------------
# single-node battery arbitrage: closed form
# --------------------------------------------------------------------------

def test_battery_arbitrage_closed_form():
    Dm, eta_k = 100.0, 30.0
    r = cases.REG_R
    net = cases.Network(
        n_nodes=1, line_from=np.zeros(0, np.int32), line_to=np.zeros(0, np.int32),
        line_beta=np.zeros(0), gen_node=np.zeros(2, np.int32),
        gen_kind=np.array([cases.SOLAR, cases.GAS], np.int32),
        gen_cost=np.array([20.0, 60.0]), gen_emis=np.array([0.0, 0.4]),
        batt_node=np.zeros(1, np.int32),
        eta_min=np.array([500.0, 500.0, eta_k]), eta_max=np.array([900.0, 900.0, 4 * eta_k]),
        gamma=np.full(3, 1e5))
    sc = cases.Scenario(network=0, T=2, avail=np.array([[1.0, 0.0], [1.0, 1.0]]),
                        load=np.array([[Dm, Dm]]), weight=4380.0)
    cs = cases.Case(name="arb", networks=[net], scenarios=[sc])
    qp, sol = _solve(cs)
    vs = qp.dims["vs"]
    ch, dis, soc = sol.x[vs["ch"]], sol.x[vs["dis"]], sol.x[vs["soc"]]
    np.testing.assert_allclose(ch, [eta_k, 0.0], atol=1e-8)
    np.testing.assert_allclose(dis, [0.0, 0.95 * eta_k], atol=1e-8)
    np.testing.assert_allclose(soc, [0.95 * eta_k, 0.0], atol=1e-8)
    e = eta_k
    dV = 20 - 0.95 * 60 + r * ((Dm + e) - 0.95 * (Dm - 0.95 * e) + e + 2 * 0.9025 * e)
    gr = Gm.scenario_gradient(qp, sol, 0.0)
    assert abs(gr["grad"][2] - dV) < 1e-7


# --------------------------------------------------------------------------
# brute force over active sets on tiny instances
# --------------------------------------------------------------------------

def _brute_force(qp):
    n = qp.n
    E = qp.E.toarray()
    lo, hi, q, r, e = qp.lo, qp.hi, qp.q, qp.r, qp.e
    choices = []
    for i in range(n):
        c = ["free"]
        if np.isfinite(lo[i]):
            c.append("lo")
        if np.isfinite(hi[i]) and hi[i] != lo[i]:
            c.append("hi")
        if np.isfinite(lo[i]) and np.isfinite(hi[i]) and hi[i] == lo[i]:
            c = ["lo"]
        choices.append(c)
    found = []
    xs = 1.0 + np.abs(np.concatenate([lo[np.isfinite(lo)], hi[np.isfinite(hi)]])).max()
    for assign in itertools.product(*choices):
        a = np.array(assign)
        F = a == "free"
        xA = np.where(a == "lo", lo, np.where(a == "hi", hi, 0.0))
        nf = int(F.sum())
        m = E.shape[0]
        EF = E[:, F]
        Kmat = np.block([[r * np.eye(nf), -EF.T], [EF, np.zeros((m, m))]])
        rhs = np.concatenate([-q[F], e - E[:, ~F] @ xA[~F]])
        sol, *_ = np.linalg.lstsq(Kmat, rhs, rcond=None)
        if np.abs(Kmat @ sol - rhs).max() > 1e-7 * (1 + np.abs(rhs).max()):
            continue
        x = xA.copy()
        x[F] = sol[:nf]
        y = sol[nf:]
        if np.any(x < lo - 1e-9 * xs) or np.any(x > hi + 1e-9 * xs):
            continue
        z = E.T @ y - q - r * x
        tolz = 1e-7 * (1 + np.abs(q).max())
        if np.any(z[a == "hi"] < -tolz) or np.any(z[(a == "lo") & (lo != hi)] > tolz):
            continue
        found.append(x)
    return found


@pytest.mark.parametrize("seed,kw", [
    (1, dict(n_nodes=2, G=2, B=1, T=1)),
    (2, dict(n_nodes=2, G=2, B=0, T=2)),
    (3, dict(n_nodes=1, G=1, B=1, T=2, with_line=False)),
    (4, dict(n_nodes=2, G=1, B=1, T=1)),
])
def test_brute_force_tiny(seed, kw):
    cs = cases.tiny_random(seed, **kw)
    eta = cs.eta_min()
    qp, sol = _solve(cs, eta)
    found = _brute_force(qp)
    assert len(found) >= 1
    for x in found:          # x* is unique (strongly convex): all KKT points agree
        np.testing.assert_allclose(x, found[0], atol=1e-6)
    np.testing.assert_allclose(sol.x, found[0], atol=1e-6)
    V = 0.5 * qp.r * found[0] @ found[0] + qp.q @ found[0]
    assert abs(sol.obj - V) <= 1e-9 * max(1.0, abs(V))


# --------------------------------------------------------------------------
# certificates, envelope identity, finite differences, invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mk", [cases.config0, lambda: cases.small_geo(omega=50.0)])
def test_kkt_certificate_and_weak_duality(mk):
    cs = mk()
    qp, sol = _solve(cs)
    res = D.kkt_residual(qp, sol.x, sol.y)
    assert res["kkt"] <= 1e-9
    assert res["P"] - res["D"] >= -1e-9 * abs(res["P"])
    # D(y) is a lower bound for any y: perturbed duals give lower values
    rng = np.random.default_rng(0)
    for _ in range(3):
        yp = sol.y + rng.normal(0, 1.0, size=sol.y.shape)
        assert D.dual_function(qp, yp) <= res["P"] + 1e-6 * abs(res["P"])


def test_envelope_identity_and_sign():
    cs = cases.config0()
    eta = cases.jitter(cs.eta_min(), 3, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    qp = D.assemble(cs, 0, eta)
    sol = D.solve(qp)
    gr = Gm.scenario_gradient(qp, sol, 0.0)
    scale = np.abs(gr["grad"]).max()
    assert np.abs(gr["grad"] - gr["envelope"]).max() <= 1e-9 * scale
    # the operating cost never increases with more capacity
    assert np.all(gr["grad"] <= 1e-9 * scale)


@pytest.mark.parametrize("omega", [0.0, 50.0])
def test_gradient_matches_central_differences(omega):
    cs = cases.config0()
    eta = cases.jitter(cs.eta_min(), 5, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    qp = D.assemble(cs, 0, eta)
    sol = D.solve(qp)
    gr = Gm.scenario_gradient(qp, sol, omega)
    g = gr["grad"]
    for j in range(qp.K):
        fd = Gm.central_difference(cs, 0, eta, j, omega, h=1e-3)
        if abs(fd["forward"] - fd["backward"]) > 1e-3 * max(1.0, abs(fd["central"])) + 1.0:
            continue   # kink along this coordinate
        assert abs(g[j] - fd["central"]) <= 1e-5 * np.abs(g).max() + 1e-3, (j, g[j], fd)


def test_value_convex_in_capacity():
    cs = cases.config0()
    eta = cs.eta_min().copy()
    h = 5.0
    for j in [0, 2, 12, 20]:
        ep, em = eta.copy(), eta.copy()
        ep[j] += h
        em[j] = max(em[j] - h, 0.0)
        v0 = Gm.value(cs, 0, eta, 0.0)
        vp = Gm.value(cs, 0, ep, 0.0)
        vm = Gm.value(cs, 0, em, 0.0)
        assert vp <= v0 + 1e-6 * abs(v0) and v0 <= vm + 1e-6 * abs(v0)
        assert vp + vm - 2 * v0 >= -1e-6 * abs(v0)


def test_hours_separate_without_batteries():
    cs = cases.small_geo(n_nodes=8, G=16, B=0, T=4, S=1, seed=11)
    qp, sol = _solve(cs)
    net = cs.networks[0]
    sc = cs.scenarios[0]
    total = 0.0
    for t in range(sc.T):
        one = cases.Case(name="h", networks=[net], scenarios=[cases.Scenario(
            network=0, T=1, avail=sc.avail[:, t:t + 1], load=sc.load[:, t:t + 1], weight=8760.0)])
        _, s1 = _solve(one)
        total += s1.obj
    assert abs(total - sol.obj) <= 1e-8 * abs(sol.obj)


def test_battery_energy_conservation_and_recursion():
    cs = cases.config0()
    qp, sol = _solve(cs)
    vs = qp.dims["vs"]
    T = qp.dims["T"]
    ch = sol.x[vs["ch"]].reshape(-1, T)
    dis = sol.x[vs["dis"]].reshape(-1, T)
    soc = sol.x[vs["soc"]].reshape(-1, T)
    # cyclic horizon: charged energy after losses equals discharged energy
    np.testing.assert_allclose((0.95 * ch - dis).sum(1), 0.0, atol=1e-7)
    np.testing.assert_allclose(soc, np.roll(soc, 1, axis=1) + 0.95 * ch - dis, atol=1e-7)


def test_system_balance_and_flow_physics():
    cs = cases.config0()
    qp, sol = _solve(cs)
    vs = qp.dims["vs"]
    T = qp.dims["T"]
    net = cs.networks[0]
    inj = (sol.x[vs["p"]].reshape(-1, T).sum(0) + sol.x[vs["u"]].reshape(-1, T).sum(0)
           + (sol.x[vs["dis"]] - sol.x[vs["ch"]]).reshape(-1, T).sum(0))
    np.testing.assert_allclose(inj, cs.scenarios[0].load.sum(0), rtol=1e-9)
    th = sol.x[vs["th"]].reshape(-1, T)
    f = sol.x[vs["f"]].reshape(-1, T)
    np.testing.assert_allclose(f, net.line_beta[:, None] * (th[net.line_from] - th[net.line_to]), atol=1e-7)


def test_zero_capacity_line_decouples():
    cs = cases.two_node(20.0, 60.0, 300.0, 200.0, 150.0, 80.0, 10.0)
    eta = cs.eta_min().copy()
    eta[2] = 0.0
    qp, sol = _solve(cs, eta)
    vs = qp.dims["vs"]
    assert abs(sol.x[vs["f"]][0]) < 1e-9
    # node B alone: expensive unit serves the whole load
    assert abs(sol.x[vs["p"]][1] - 150.0) < 1e-6
