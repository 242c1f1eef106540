"""Write full-size oracle reference values for the GPU parity tests.

Calls only ``oracle/`` (and the seeded input generator).  For each listed
configuration and scenario it solves the dispatch QP with the FP64 interior
point + polish at capacities eta_min jittered by U[0, 1e-2] MW (seed 11),
and stores the objective, the emissions and the per-scenario capacity
gradient of h_s (not weighted) as JSON:

    python tests/golden/make_golden.py 1 0 1      # config 1, scenarios 0 and 1
    python tests/golden/make_golden.py 3 0        # config 3, scenario 0
    python tests/golden/make_golden.py --spread 1 0   # add the kink spread to a stored file
    python tests/golden/make_golden.py --spread-draw 3 1 0   # one draw of it (draws run in parallel)

The spread is the largest relative change of the oracle gradient when every
capacity moves by U[-0.02, 0.02] MW (two draws): the GPU solves to a balance
residual of about that size, so near a kink of the piecewise-affine dispatch
map its gradient cannot be more accurate than this.  The moved gradients are
stored too, so a test can take the same measure on any subset of capacities.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2410_13055_amd import cases  # noqa: E402
from oracle import dispatch as D  # noqa: E402
from oracle import gradient as Gm  # noqa: E402

JITTER_SEED = 11


def golden_eta(case):
    return cases.jitter(case.eta_min(), JITTER_SEED, eta_min=case.eta_min(), eta_max=case.eta_max())


SPREAD_MW = 0.02


def spread(cfg, s):
    case = cases.by_id(cfg)
    eta = golden_eta(case)
    off = case.eta_offsets()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_config{cfg}_s{s}.json")
    with open(path) as fh:
        out = json.load(fh)
    g0 = np.array(out["grad"])
    net = case.scenarios[s].network
    worst = 0.0
    moved = []
    for k in range(2):
        rng = np.random.Generator(np.random.PCG64(1000 + k))
        ep = np.clip(eta + rng.uniform(-SPREAD_MW, SPREAD_MW, size=eta.shape), case.eta_min(), case.eta_max())
        qp = D.assemble(case, s, ep[off[net]:off[net + 1]])
        sol = D.solve(qp)
        g = Gm.scenario_gradient(qp, sol, case.omega)["grad"]
        moved.append([float(v) for v in g])
        worst = max(worst, float(np.linalg.norm(g - g0) / np.linalg.norm(g0)))
    out["grad_spread"] = worst
    out["spread_grads"] = moved
    out["spread_mw"] = SPREAD_MW
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"config {cfg} scenario {s}: gradient spread {worst:.2e}", flush=True)


def spread_draw(cfg, s, k):
    """One draw k of the spread, merged into the stored file under a lock
    (several draws can run as separate processes).  The lock file is left in
    place: removing it would let a process still waiting on the old file and
    a newcomer on a fresh one both hold "the" lock."""
    import fcntl
    case = cases.by_id(cfg)
    eta = golden_eta(case)
    off = case.eta_offsets()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_config{cfg}_s{s}.json")
    net = case.scenarios[s].network
    rng = np.random.Generator(np.random.PCG64(1000 + k))
    ep = np.clip(eta + rng.uniform(-SPREAD_MW, SPREAD_MW, size=eta.shape), case.eta_min(), case.eta_max())
    qp = D.assemble(case, s, ep[off[net]:off[net + 1]])
    g = Gm.scenario_gradient(qp, D.solve(qp), case.omega)["grad"]
    with open(path + ".lock", "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        with open(path) as fh:
            out = json.load(fh)
        g0 = np.array(out["grad"])
        draws = dict(out.get("spread_draws", {}))
        draws[str(k)] = [float(v) for v in g]
        out["spread_draws"] = draws
        out["spread_grads"] = [draws[d] for d in sorted(draws)]
        out["grad_spread"] = max(float(np.linalg.norm(np.array(v) - g0) / np.linalg.norm(g0))
                                 for v in out["spread_grads"])
        out["spread_mw"] = SPREAD_MW
        with open(path, "w") as fh:
            json.dump(out, fh)
    print(f"config {cfg} scenario {s} draw {k}: gradient spread so far {out['grad_spread']:.2e}", flush=True)


def main():
    if sys.argv[1] == "--spread-draw":
        spread_draw(int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4]))
        return
    if sys.argv[1] == "--spread":
        for s in sys.argv[3:] or ["0"]:
            spread(int(sys.argv[2]), int(s))
        return
    cfg = int(sys.argv[1])
    scen = [int(s) for s in sys.argv[2:]] or [0]
    case = cases.by_id(cfg)
    eta = golden_eta(case)
    off = case.eta_offsets()
    for s in scen:
        t0 = time.time()
        net = case.scenarios[s].network
        qp = D.assemble(case, s, eta[off[net]:off[net + 1]])
        sol = D.solve(qp)
        res = D.kkt_residual(qp, sol.x, sol.y)
        gr = Gm.scenario_gradient(qp, sol, case.omega)
        out = {
            "config": cfg, "scenario": s, "omega": case.omega, "jitter_seed": JITTER_SEED,
            "cost": D.primal_objective(qp, sol.x), "emis": float(qp.emis @ sol.x),
            "h": D.planner_objective(qp, sol.x, case.omega), "kkt": res["kkt"],
            "polished": bool(sol.polished), "kink": bool(gr["kink"]),
            "grad": [float(v) for v in gr["grad"]], "seconds": time.time() - t0,
        }
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_config{cfg}_s{s}.json")
        with open(path, "w") as fh:
            json.dump(out, fh)
        print(f"config {cfg} scenario {s}: cost {out['cost']:.6e} kkt {res['kkt']:.1e} "
              f"polished {sol.polished} kink {gr['kink']} {out['seconds']:.0f} s", flush=True)


if __name__ == "__main__":
    main()
