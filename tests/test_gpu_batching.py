"""Uneven batches, the two sweep forms and the autotuner (the batching row of
the hot path): results do not depend on how the work is launched."""
import numpy as np
import pytest

from paper_2410_13055_amd import cases
from oracle import dispatch as D

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _plan(case, **kw):
    from paper_2410_13055_amd import gridplan as gpb
    print(f"\n[gpu] plan {case.name} S={len(case.scenarios)} opts={kw}", flush=True)
    return gpb.Plan(case, gpb.options(**kw), stream=gpb.current_stream())


def test_tile_grid_and_work_queue_agree_bitwise():
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=2, seed=7)
    eta = cases.jitter(cs.eta_min(), 4, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    out = []
    for variant in (1, 2):
        with _plan(cs, variant=variant, block=256, check_every=64) as p:
            p.solve(eta, [0, 1])
            out.append(p.solution(1))
            assert p.tuning()[1] == variant
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_autotuner_choice_is_valid_and_does_not_change_the_answer():
    cs = cases.config0()
    eta = cases.jitter(cs.eta_min(), 1, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    qp = D.assemble(cs, 0, eta)
    ref = D.solve(qp).obj
    with _plan(cs) as p:
        cost, st, rc = p.solve(eta, [0])
        block, variant, ce, tab = p.tuning()
    assert block in (128, 256, 512) and variant in (1, 2) and ce in (32, 64, 128)
    assert np.all(tab > 0)
    assert rc == 0 and abs(cost[0] - ref) <= TOL * abs(ref)


def test_uneven_64_scenarios_in_one_batch():
    """64 scenarios with 100-500 nodes and 24/72/168-hour horizons solved as
    one batch; the oracle certifies every returned pair from its KKT residual
    and exact dual function, and re-solves the two smallest scenarios."""
    cs = cases.config2()
    S = len(cs.scenarios)
    eta = cases.jitter(cs.eta_min(), 2, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    off = cs.eta_offsets()
    with _plan(cs) as p:
        cost, st, rc = p.solve(eta, list(range(S)))
        assert rc == 0, [s for s in st if s["status"]]
        sizes = [cs.networks[s].n_nodes * cs.scenarios[s].T for s in range(S)]
        small = list(np.argsort(sizes)[:2])
        check = sorted(set(small + list(range(0, S, 8))))
        sols = {s: p.solution(int(s)) for s in check}
    for s in check:
        qp = D.assemble(cs, int(s), eta[off[s]:off[s + 1]])
        x, y = sols[s]
        res = D.kkt_residual(qp, x.astype(np.float64), y)
        assert res["kkt"] <= 1.05 * TOL, (s, res)
        assert res["P"] - res["D"] <= TOL * (1 + abs(res["P"]))
        if s in small:
            ref = D.solve(qp).obj
            assert abs(cost[s] - ref) <= TOL * abs(ref), (s, cost[s], ref)
