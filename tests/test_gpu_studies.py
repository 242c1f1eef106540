"""The two planning studies built on the hot path, small enough to check
against the oracle:

- the plan-level warm start (Section 3.2): re-planning under another carbon
  weight, started from the plan found under the first, reaches the loss of
  the cold run; the objective at the cold plan matches the oracle's;
- the key-day study (Section 3.1): stochastic batches drawn from the key
  days or from every day, each plan scored on every day; the library's
  all-day score matches the oracle's at the same capacities.
"""
import numpy as np
import pytest

from paper_2410_13055_amd import cases
from oracle import plan as OP

pytestmark = pytest.mark.gpu


def _plan(case, **kw):
    from paper_2410_13055_amd import gridplan as gpb
    print(f"\n[gpu] plan {case.name} S={len(case.scenarios)} opts={kw}", flush=True)
    return gpb.Plan(case, gpb.options(**kw), stream=gpb.current_stream())


def _phi(p, case, eta, scen, omega):
    p.solve(eta, scen, warm=1)
    return float(case.gamma() @ eta + p.objective(scen, omega, eta=eta))


def test_plan_level_warm_start_reaches_the_cold_loss_sooner():
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=4, seed=7)
    scen = list(range(4))
    lo, hi = cs.eta_min(), cs.eta_max()
    gamma = cs.gamma()
    with _plan(cs, tol=1e-5, block=256, variant=1, check_every=64) as p:
        p.solve(lo, scen)
        g0, _, _ = p.grad(scen, 200.0)
        alpha = 0.1 * float((hi - lo).min()) / float(np.abs(gamma + g0).max())

        def run(eta0, omega, steps, target=None):
            eta = eta0.copy()
            curve = [_phi(p, cs, eta, scen, omega)]
            for k in range(1, steps + 1):
                eta, _, _, rc = p.step(alpha / np.sqrt(k), scen, gamma, eta, omega=omega, warm=1)
                assert rc == 0
                curve.append(_phi(p, cs, eta, scen, omega))
                if target is not None and curve[-1] <= target:
                    break
            return eta, curve

        src, _ = run(lo, 200.0, 40)
        eta_c, cold = run(lo, 150.0, 60)
        best = min(cold)
        kc = next(k for k, v in enumerate(cold) if v <= 1.02 * best)
        eta_w, warm = run(src, 150.0, 60, target=1.02 * best)
        kw = next((k for k, v in enumerate(warm) if v <= 1.02 * best), None)
        print(f"[gpu] plan-level warm start: cold {kc} steps, warm {kw} steps to within 2 % of {best:.6e}",
              flush=True)
        assert kw is not None
        phi_gpu = _phi(p, cs, eta_c, scen, 150.0)
    phi_orc = OP.phi(cs, eta_c, scen, 150.0)[0]
    assert abs(phi_gpu - phi_orc) <= 1e-4 * abs(phi_orc)


def test_key_day_sampling_and_all_day_scoring():
    cs = cases.year(n_nodes=12, G=30, B=3, days=24, omega=200.0)
    days = list(range(24))
    lo = cs.eta_min()
    gamma = cs.gamma()
    kd = cases.key_days(cs, lo, per=2)
    assert len(kd) == 8
    with _plan(cs, tol=1e-5, block=256, variant=1, check_every=64) as p:
        p.solve(lo, kd[:4])
        g0, _, _ = p.grad(kd[:4], cs.omega)
        alpha = 0.1 * float((cs.eta_max() - lo).min()) / float(np.abs(gamma + g0).max())
        scores = {}
        for label, pool, seed in (("key days", kd, 1), ("all days", days, 2)):
            rng = np.random.default_rng(seed)
            eta = lo.copy()
            for k in range(1, 4):
                batch = sorted(rng.choice(pool, 4, replace=False).tolist())
                assert set(batch) <= set(pool)
                eta, _, _, rc = p.step(alpha / np.sqrt(k), batch, gamma, eta, omega=cs.omega, warm=1)
                assert rc == 0
            scores[label] = (eta, _phi(p, cs, eta, days, cs.omega))
    for label, (eta, phi_gpu) in scores.items():
        phi_orc = OP.phi(cs, eta, days, cs.omega)[0]
        print(f"[gpu] {label}: all-day objective {phi_gpu:.6e} (oracle {phi_orc:.6e})", flush=True)
        assert abs(phi_gpu - phi_orc) <= 1e-4 * abs(phi_orc)
