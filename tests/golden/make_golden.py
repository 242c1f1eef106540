"""Write full-size oracle reference values for the GPU parity tests.

Calls only ``oracle/`` (and the seeded input generator).  For each listed
configuration and scenario it solves the dispatch QP with the FP64 interior
point + polish at capacities eta_min jittered by U[0, 1e-2] MW (seed 11) and
stores, as JSON:

- the objective, the emissions and the planner objective h_s;
- the per-scenario capacity gradient of h_s (not weighted by w_s), from the
  least-squares adjoint (Section 2.2, implicit function theorem);
- for every capacity, the central difference of h_s with h = 1e-3 MW from the
  fixed-active-set re-solve (one factorisation, two back-solves per capacity)
  and whether both ends verified as optimal ("fd_ok"); a coordinate that does
  not verify has a kink of the piecewise-affine dispatch map within 1e-3 MW
  and carries no derivative there;
- the same verification over +-0.05 MW ("ok_wide");
- per capacity, the distance to the nearest kink along it ("kink_distance",
  MW, from a ratio test on the fixed-active-set step) and the curvature of
  h_s along it ("curvature"): a solve whose duality gap is G determines the
  derivative of a convex h_s only to within G / distance + curvature *
  distance / 2;
- a stratified 20-capacity subset among the verified coordinates: 8
  generators (3 gas, 3 solar, 2 wind), the 8 lines with the largest gradient
  magnitude (congested), 4 batteries.

    python tests/golden/make_golden.py 1 0 1      # config 1, scenarios 0 and 1
    python tests/golden/make_golden.py 3 1        # config 3, scenario 1 (subset mode)
    python tests/golden/make_golden.py 3 0 --all  # config 3, differences on every capacity

For the 500-node workload (config 3) a back-solve of the reduced system costs
seconds, so the differences are taken on 40 stratified candidates only (12
generators, the 16 lines with the largest gradient magnitude, 12 batteries),
from which the 20-capacity subset is drawn among the verified ones; the
per-coordinate arrays then hold NaN / 0 elsewhere.

The interior-point solution of each scenario is cached (uncompressed npz,
not committed) under tests/golden/.cache/, so the derived values can be
recomputed without the solve: a config-3 solve takes hours of CPU.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2410_13055_amd import cases  # noqa: E402
from oracle import dispatch as D  # noqa: E402
from oracle import gradient as Gm  # noqa: E402

JITTER_SEED = 11
FD_H = 1e-3
WIDE_H = 0.05


def golden_eta(case):
    return cases.jitter(case.eta_min(), JITTER_SEED, eta_min=case.eta_min(), eta_max=case.eta_max())


def _solution(case, cfg, s, qp):
    """Polished oracle solution of scenario s, from the cache when present."""
    cdir = os.path.join(HERE, ".cache")
    path = os.path.join(cdir, f"config{cfg}_s{s}.npz")
    if os.path.exists(path):
        z = np.load(path)
        sol = D.Solution(x=z["x"], y=z["y"], z=z["z"], obj=float(z["obj"]), iters=int(z["iters"]),
                         status=str(z["status"]), history=[], polished=bool(z["polished"]),
                         degenerate=bool(z["degenerate"]), active_lo=z["active_lo"], active_hi=z["active_hi"])
        return sol, True
    sol = D.solve(qp)
    os.makedirs(cdir, exist_ok=True)
    np.savez(path, x=sol.x, y=sol.y, z=sol.z, obj=sol.obj, iters=sol.iters, status=sol.status,
             polished=sol.polished, degenerate=sol.degenerate, active_lo=sol.active_lo, active_hi=sol.active_hi)
    return sol, False


def candidates40(case, grad):
    """Stratified candidates for the subset mode: 4 generators of each kind,
    the 16 lines with the largest gradient magnitude, 12 batteries."""
    net = case.networks[0]
    G, L = net.n_gens, net.n_lines
    rng = np.random.default_rng(40)
    idx = []
    for kind in (cases.GAS, cases.SOLAR, cases.WIND):
        idx += [int(v) for v in rng.choice(np.where(net.gen_kind == kind)[0], 4, replace=False)]
    idx += [int(G + v) for v in np.argsort(-np.abs(grad[G:G + L]))[:16]]
    idx += [int(G + L + v) for v in rng.choice(net.n_batt, 12, replace=False)]
    return np.array(idx)


def subset20(case, grad, ok):
    """Stratified 20-capacity subset among the coordinates in ``ok``."""
    net = case.networks[0]
    G, L = net.n_gens, net.n_lines
    rng = np.random.default_rng(20)
    idx = []
    for kind, n in ((cases.GAS, 3), (cases.SOLAR, 3), (cases.WIND, 2)):
        cand = np.where((net.gen_kind == kind) & ok[:G])[0]
        idx += [int(v) for v in rng.choice(cand, n, replace=False)]
    lines = np.where(ok[G:G + L])[0]
    idx += [int(G + v) for v in lines[np.argsort(-np.abs(grad[G + lines]))[:8]]]
    bat = np.where(ok[G + L:])[0]
    idx += [int(G + L + v) for v in rng.choice(bat, 4, replace=False)]
    return idx


def main():
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    every = "--all" in sys.argv   # differences on every capacity even for config 3
    cfg = int(args[0])
    scen = [int(s) for s in args[1:]] or [0]
    case = cases.by_id(cfg)
    eta = golden_eta(case)
    off = case.eta_offsets()
    for s in scen:
        t0 = time.time()
        net = case.scenarios[s].network
        qp = D.assemble(case, s, eta[off[net]:off[net + 1]])
        sol, cached = _solution(case, cfg, s, qp)
        t_solve = time.time() - t0
        res = D.kkt_residual(qp, sol.x, sol.y)
        gr = Gm.scenario_gradient(qp, sol, case.omega)
        subset_mode = cfg == 3 and not every
        js = candidates40(case, gr["grad"]) if subset_mode else None
        fd_s = Gm.fixed_set_differences(qp, sol, case.omega, h=FD_H, js=js)
        wide_s = Gm.fixed_set_differences(qp, sol, case.omega, h=WIDE_H, js=js)

        def full(vals, fill):
            if not subset_mode:
                return np.asarray(vals)
            out = np.full(qp.K, fill, dtype=np.asarray(vals).dtype)
            out[js] = vals
            return out
        fd = {k: full(fd_s[k], np.nan if k in ("central", "dist", "curv") else False)
              for k in ("central", "ok", "dist", "curv")}
        wide = {"ok": full(wide_s["ok"], False)}
        ok = fd["ok"]
        scale = np.abs(gr["grad"]).max()
        agree = float(np.abs(fd["central"][ok] - gr["grad"][ok]).max(initial=0.0) / scale)
        out = {
            "config": cfg, "scenario": s, "omega": case.omega, "jitter_seed": JITTER_SEED,
            "cost": D.primal_objective(qp, sol.x), "emis": float(qp.emis @ sol.x),
            "h": D.planner_objective(qp, sol.x, case.omega), "kkt": res["kkt"],
            "polished": bool(sol.polished), "rank_deficient": bool(gr["rank_deficient"]),
            "grad": [float(v) for v in gr["grad"]],
            "fd_h": FD_H, "fd_central": [float(v) for v in fd["central"]],
            "fd_candidates": None if js is None else [int(v) for v in js],
            "fd_ok": [int(v) for v in ok], "ok_wide": [int(v) for v in wide["ok"]], "wide_h": WIDE_H,
            "kink_distance": [float(v) for v in fd["dist"]], "curvature": [float(v) for v in fd["curv"]],
            "fd_vs_grad_max_rel": agree,
            "subset20": subset20(case, gr["grad"], ok),
            "solve_seconds": t_solve if not cached else None, "seconds": time.time() - t0,
        }
        path = os.path.join(HERE, f"oracle_config{cfg}_s{s}.json")
        with open(path, "w") as fh:
            json.dump(out, fh)
        print(f"config {cfg} scenario {s}: cost {out['cost']:.6e} kkt {res['kkt']:.1e} "
              f"polished {sol.polished} kinks within {FD_H} MW: {int((~ok).sum())} of {qp.K}, within "
              f"{WIDE_H} MW: {int((~wide['ok']).sum())}; fd vs grad {agree:.1e}; {out['seconds']:.0f} s"
              f"{' (cached solve)' if cached else ''}", flush=True)


if __name__ == "__main__":
    main()
