"""The seeded input generator: determinism, the workload sizes of the hot
path, and the shape rules every generated case satisfies."""
import numpy as np
import pytest

from paper_2410_13055_amd import cases


def _arrays(cs):
    out = []
    for n in cs.networks:
        out += [n.line_from, n.line_to, n.line_beta, n.gen_node, n.gen_cost, n.eta_min, n.eta_max, n.gamma]
    for sc in cs.scenarios:
        out += [sc.avail, sc.load]
    return out


@pytest.mark.parametrize("make", [cases.config0, lambda **k: cases.config1(S=2, **k),
                                  lambda **k: cases.config2(S=3, **k)])
def test_same_seed_same_case_other_seed_other_case(make):
    a, b, c = make(), make(), make(seed=12345)
    for x, y in zip(_arrays(a), _arrays(b)):
        np.testing.assert_array_equal(x, y)
    assert any(x.shape != z.shape or not np.array_equal(x, z) for x, z in zip(_arrays(a), _arrays(c)))


@pytest.mark.parametrize("cfg,nx,ny,K", [(0, 912, 384, 22), (1, 359520, 117600, 1460)])
def test_workload_sizes(cfg, nx, ny, K):
    """Per-scenario variable and equality counts of the workload table:
    n_x = (G + L + 2N + 3B) T, n_eq = (N + L + B) T, K = G + L + B."""
    cs = cases.by_id(cfg, S=1) if cfg else cases.config0()
    n = cs.networks[0]
    T = cs.scenarios[0].T
    assert (n.n_gens + n.n_lines + 2 * n.n_nodes + 3 * n.n_batt) * T == nx
    assert (n.n_nodes + n.n_lines + n.n_batt) * T == ny
    assert cs.K == K


def test_generated_values_respect_their_ranges():
    cs = cases.config1(S=2)
    n = cs.networks[0]
    assert np.all((n.line_beta >= 5) & (n.line_beta <= 20))
    assert np.all(n.eta_max >= n.eta_min) and np.all(n.eta_min >= 0)
    for sc in cs.scenarios:
        assert np.all((sc.avail >= 0) & (sc.avail <= 1))
        assert np.all(sc.load > 0)
        # every value is exactly representable in FP32 (both paths read the same numbers)
        np.testing.assert_array_equal(sc.load, sc.load.astype(np.float32).astype(np.float64))
    # connected: a breadth-first search from node 0 reaches every node
    adj = [[] for _ in range(n.n_nodes)]
    for a, b in zip(n.line_from, n.line_to):
        adj[a].append(b)
        adj[b].append(a)
    seen, stack = {0}, [0]
    while stack:
        for m in adj[stack.pop()]:
            if m not in seen:
                seen.add(m)
                stack.append(m)
    assert len(seen) == n.n_nodes


def test_key_days_follow_their_definition():
    """Key days (Section 3.1 footnote): 4 days each of highest peak load,
    highest peak net load, highest peak renewable availability and lowest
    renewable energy, distinct, 16 in all; a year has seasons (summer load
    above winter load on average)."""
    cs = cases.year(n_nodes=12, G=30, B=3, days=48)
    eta = cs.eta_min()
    kd = cases.key_days(cs, eta)
    assert len(kd) == 16 == len(set(kd))
    net = cs.networks[0]
    ren = net.gen_cost == 0
    load = np.array([sc.load.sum(0) for sc in cs.scenarios])
    renew = np.array([(sc.avail[ren] * eta[:net.n_gens][ren, None]).sum(0) for sc in cs.scenarios])
    # the four highest peak-load days are always chosen (their criterion goes first)
    assert set(np.argsort(-load.max(1))[:4].tolist()) <= set(kd)
    # every criterion has at least its four best days among the chosen or
    # already taken by an earlier criterion
    for col in ((load - renew).max(1), renew.max(1), -renew.sum(1)):
        best = np.argsort(-col)
        k = 0
        for s in best:
            if s in kd:
                k += 1
            if k == 4:
                break
        assert k == 4
    mid = [d for d in range(48) if 18 <= d < 30]
    ends = [d for d in range(48) if d < 6 or d >= 42]
    assert load[mid].mean() > load[ends].mean()
