"""GPU planning layer: full-size parity against stored oracle values, the
autograd bridge, and a 10-step projected-gradient run whose every step is
checked against the oracle gradient at the GPU's current capacities
(Section 2.2).

Gradient bar: relative 2-norm error <= max(1e-3, spread), where spread is how
much the oracle's own gradient moves when every capacity moves by up to
0.02 MW, the GPU's balance-residual resolution at a 1e-4 KKT residual.  The
dispatch map is piecewise affine; near one of its kinks (for example a node
whose unserved load is within that resolution of zero, where the price jumps
between the marginal cost and the penalty) no solution of that accuracy
determines the gradient more closely."""
import json
import os

import numpy as np
import pytest

from paper_2410_13055_amd import cases
from oracle import dispatch as D
from oracle import gradient as Gm

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-4
SPREAD_MW = 0.02


def _spread(case, s, eta, omega, g0, draws=2):
    """Largest relative change of the oracle gradient of scenario s under
    capacity moves of up to SPREAD_MW."""
    off = case.eta_offsets()
    net = case.scenarios[s].network
    worst = 0.0
    for k in range(draws):
        rng = np.random.Generator(np.random.PCG64(1000 + k))
        ep = np.clip(eta + rng.uniform(-SPREAD_MW, SPREAD_MW, size=eta.shape), case.eta_min(), case.eta_max())
        qp = D.assemble(case, s, ep[off[net]:off[net + 1]])
        g = Gm.scenario_gradient(qp, D.solve(qp), omega)["grad"]
        worst = max(worst, float(np.linalg.norm(g - g0) / np.linalg.norm(g0)))
    return worst


def _plan(case, **kw):
    from paper_2410_13055_amd import gridplan as gpb
    print(f"\n[gpu] plan {case.name} S={len(case.scenarios)} opts={kw}", flush=True)
    return gpb.Plan(case, gpb.options(**kw), stream=gpb.current_stream())


def _golden(cfg, s):
    path = os.path.join(GOLD, f"oracle_config{cfg}_s{s}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as fh:
        return json.load(fh)


def _golden_eta(case):
    return cases.jitter(case.eta_min(), 11, eta_min=case.eta_min(), eta_max=case.eta_max())


def _subset20(case, grad):
    """8 generators (3 gas, 3 solar, 2 wind), 8 lines (the 8 with the largest
    gradient magnitude, i.e. congested), 4 batteries: a fixed, stratified
    20-capacity subset."""
    net = case.networks[0]
    G, L = net.n_gens, net.n_lines
    rng = np.random.default_rng(20)
    idx = []
    for kind, n in ((cases.GAS, 3), (cases.SOLAR, 3), (cases.WIND, 2)):
        idx += list(rng.choice(np.where(net.gen_kind == kind)[0], n, replace=False))
    idx += list(G + np.argsort(-np.abs(grad[G:G + L]))[:8])
    idx += list(G + L + rng.choice(net.n_batt, 4, replace=False))
    return np.array(idx)


@pytest.mark.parametrize("cfg,scen", [(1, [0, 1]), (3, [0, 1])])
def test_full_size_against_stored_oracle(cfg, scen):
    """Full-size scenarios against stored oracle values: cost, the full
    gradient and a 20-capacity subset of it at the 1e-4 KKT tolerance.  The
    subset picks the most congested lines, whose gradient entries follow the
    line duals; a 1e-4 solve can leave about 1 % in a single such entry
    (config 3 scenario 1: one line), which the full-vector bar absorbs and a
    20-entry subset does not.  A subset that misses its bar is therefore
    solved again to 1e-5 and must meet it there: an error that vanishes as
    the solve tightens is the solve's accuracy, one that stays is the
    gradient's."""
    golds = [_golden(cfg, s) for s in scen]
    case = cases.by_id(cfg)
    eta = _golden_eta(case)
    omega = case.omega
    with _plan(case) as p:
        cost, st, rc = p.solve(eta, scen)
        assert rc == 0, st
        grads = []
        for s in scen:
            p.solve(eta, [s], warm=1)
            g, h, _ = p.grad([s], omega)
            grads.append(g)
    for b, (s, gd) in enumerate(zip(scen, golds)):
        gap = abs(cost[b] - gd["cost"]) / abs(gd["cost"])
        assert gap <= TOL, (s, cost[b], gd["cost"])
        ref = case.scenarios[s].weight * np.array(gd["grad"])
        bar = max(1e-3, gd.get("grad_spread", 0.0))
        err = np.linalg.norm(grads[b] - ref) / np.linalg.norm(ref)
        print(f"[gpu] config {cfg} scenario {s}: grad err {err:.2e} bar {bar:.2e}", flush=True)
        assert err <= bar, (s, err, bar)
        sub = _subset20(case, ref)
        # the spread measure restricted to the subset, from the stored
        # oracle gradients at the moved capacities
        g0 = np.array(gd["grad"])
        sub_spread = max([np.linalg.norm(np.array(g)[sub] - g0[sub]) / np.linalg.norm(g0[sub])
                          for g in gd.get("spread_grads", [])] or [0.0])
        bar_sub = max(1e-3, sub_spread)
        errs = np.linalg.norm(grads[b][sub] - ref[sub]) / np.linalg.norm(ref[sub])
        print(f"[gpu] config {cfg} scenario {s}: subset grad err {errs:.2e} bar {bar_sub:.2e}", flush=True)
        if errs > bar_sub:
            with _plan(case, tol=1e-5, max_iter=2_000_000) as q:
                _, st5, rc5 = q.solve(eta, [s])
                assert rc5 == 0, st5
                g5, _, _ = q.grad([s], omega)
            errs = np.linalg.norm(g5[sub] - ref[sub]) / np.linalg.norm(ref[sub])
            print(f"[gpu] config {cfg} scenario {s}: subset grad err at 1e-5 {errs:.2e}", flush=True)
        assert errs <= bar_sub, (s, errs, bar_sub)


def test_autograd_bridge_matches_oracle_and_differences():
    import torch

    from paper_2410_13055_amd.autograd import planning_objective
    cs = cases.config0()
    omega = 50.0
    eta0 = cases.jitter(cs.eta_min(), 6, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    gamma = torch.tensor(cs.gamma(), dtype=torch.float64, device="cuda")
    with _plan(cs) as p:
        eta = torch.tensor(eta0, dtype=torch.float64, device="cuda", requires_grad=True)
        loss = planning_objective(eta, p, [0], gamma, omega)
        loss.backward()
        g = eta.grad.cpu().numpy()
    qp = D.assemble(cs, 0, eta0)
    sol = D.solve(qp)
    w = cs.scenarios[0].weight
    ref = cs.gamma() + w * Gm.scenario_gradient(qp, sol, omega)["grad"]
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) <= 1e-3
    href = cs.gamma() @ eta0 + w * D.planner_objective(qp, sol.x, omega)
    assert abs(loss.item() - href) <= TOL * abs(href)
    # central differences of the oracle on a few capacities
    for j in (0, 5, 13, 21):
        fd = Gm.central_difference(cs, 0, eta0, j, omega)
        if abs(fd["forward"] - fd["backward"]) > 1e-3 * max(1.0, abs(fd["central"])) + 1.0:
            continue
        assert abs(g[j] - (cs.gamma()[j] + w * fd["central"])) <= 1e-3 * np.abs(ref).max()


def test_ten_gradient_steps_track_the_oracle():
    cs = cases.config0()
    eta = cs.eta_min().copy()
    gamma = cs.gamma()
    with _plan(cs) as p:
        # step size of the survey's reading: 0.1 * min box width / |Delta0|_inf
        p.solve(eta, [0])
        g0, _, _ = p.grad([0])
        alpha = 0.1 * (cs.eta_max() - cs.eta_min()).min() / np.abs(gamma + g0).max()
        phis = []
        for k in range(10):
            eta_new, phi, delta, rc = p.step(alpha, [0], gamma, eta, warm=1 if k else 0)
            assert rc == 0
            qp = D.assemble(cs, 0, eta)
            sol = D.solve(qp)
            g0 = Gm.scenario_gradient(qp, sol, 0.0)["grad"]
            w = cs.scenarios[0].weight
            ref = gamma + w * g0
            err = np.linalg.norm(delta - ref) / np.linalg.norm(ref)
            # the spread of the dispatch part, expressed relative to Delta
            sp = _spread(cs, 0, eta, 0.0, g0) * np.linalg.norm(w * g0) / np.linalg.norm(ref)
            bar = max(1e-3, sp)
            print(f"[gpu] step {k}: Delta err {err:.2e} bar {bar:.2e}", flush=True)
            assert err <= bar, (k, err, bar)
            np.testing.assert_allclose(eta_new, np.clip(eta - alpha * delta, cs.eta_min(), cs.eta_max()))
            phis.append(phi)
            eta = eta_new
    assert phis[-1] < phis[0]


def test_uneven_batch_small():
    """Scenarios of different networks and horizons in one batch.  Horizons
    that are not multiples of 4 (1 and 50) take the one-hour-per-thread
    sweeps and one battery chain per block; 50 hours also exceed the chain
    inverse's tap span, 1 hour does not."""
    shapes = [(12, 24), (20, 72), (8, 1), (16, 48), (10, 50)]
    nb = len(shapes)
    nets, scens = [], []
    for i, (n, T) in enumerate(shapes):
        c = cases.small_geo(n_nodes=n, G=3 * n, B=max(1, n // 6), T=T, S=1, seed=30 + i)
        nets.append(c.networks[0])
        sc = c.scenarios[0]
        sc.network = i
        scens.append(sc)
    case = cases.Case(name="uneven_small", networks=nets, scenarios=scens)
    eta = cases.jitter(case.eta_min(), 8, eta_min=case.eta_min(), eta_max=case.eta_max())
    off = case.eta_offsets()
    with _plan(case) as p:
        cost, st, rc = p.solve(eta, list(range(nb)))
        assert rc == 0
        g, h, _ = p.grad(list(range(nb)))
        for s in range(nb):
            x, y = p.solution(s)
            qp = D.assemble(case, s, eta[off[s]:off[s + 1]])
            sol = D.solve(qp)
            assert abs(cost[s] - sol.obj) <= TOL * abs(sol.obj)
            assert D.kkt_residual(qp, x.astype(np.float64), y)["kkt"] <= 1.05 * TOL
            ref = case.scenarios[s].weight * Gm.scenario_gradient(qp, sol, 0.0)["grad"] / nb
            gs = g[off[s]:off[s + 1]]
            assert np.linalg.norm(gs - ref) / np.linalg.norm(ref) <= 1e-3


def test_cold_solves_along_a_planning_path_converge():
    """Cold solves at every iterate of a 10-step projected-gradient path on
    the tiny case converge (a weight rule that lets the duality gap push the
    primal weight down while the balance residual stalls left several of
    these stuck at a balance residual of ~0.2)."""
    cs = cases.config0()
    eta = cs.eta_min().copy()
    gamma = cs.gamma()
    with _plan(cs) as p, _plan(cs) as q:
        p.solve(eta, [0])
        g0, _, _ = p.grad([0])
        alpha = 0.1 * (cs.eta_max() - cs.eta_min()).min() / np.abs(gamma + g0).max()
        iters = []
        for k in range(10):
            eta, phi, delta, rc = p.step(alpha, [0], gamma, eta, warm=1 if k else 0)
            assert rc == 0
            _, st, rc = q.solve(eta, [0], warm=0)
            assert rc == 0, (k, st)
            iters.append(st[0]["iters"])
    print(f"\n[gpu] cold iterations along the path: {iters}", flush=True)


def test_adjoint_solves_along_a_carbon_priced_planning_path_converge():
    """14 projected-SGD steps at 150 $/t on the 100-node case (batches of 4 of
    16 scenarios, step alpha/sqrt(k)): every dispatch and adjoint solve
    converges.  Under a primal-weight rule for the adjoint that balanced the
    weighted primal and dual movement, the adjoint of steps 8 and 13
    diverged (KKT residual growing to 1e6)."""
    cs = cases.geo100()
    pool = list(range(16))
    lo, hi = cs.eta_min(), cs.eta_max()
    gamma = cs.gamma()
    omega = 150.0
    with _plan(cs, block=256, variant=1, check_every=64) as p:
        p.solve(lo, pool[:4], warm=0)
        g0, _, _ = p.grad(pool[:4], 200.0)
        alpha = 0.1 * float((hi - lo).min()) / float(np.abs(gamma + g0).max())
        p.solve(lo, pool, warm=1)
        rng = np.random.default_rng(int(omega))
        eta = lo.copy()
        for k in range(1, 15):
            scen = sorted(rng.choice(pool, 4, replace=False).tolist())
            _, st, rc = p.solve(eta, scen, warm=1)
            assert rc == 0, (k, st)
            g, _, rc2 = p.grad(scen, omega)
            assert rc2 == 0, k
            assert np.abs(g).max() < 1e9, (k, np.abs(g).max())
            eta = np.clip(eta - alpha / np.sqrt(k) * (gamma + g), lo, hi)
            if k % 5 == 0:
                p.solve(eta, pool, warm=1)
