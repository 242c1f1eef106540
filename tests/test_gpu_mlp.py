"""The learned warm start on the GPU: BF16 MFMA GEMMs and the network's
forward/backward against the FP64 reference that rounds at the same points,
feature and target extraction against the oracle, seeding, and what a
trained network gains over a cold start."""
import numpy as np
import pytest

from paper_2410_13055_amd import cases
from oracle import dispatch as D
from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _gb():
    from paper_2410_13055_amd import gridplan
    return gridplan


@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
@pytest.mark.parametrize("M_,N_,K_", [(200, 130, 70), (1, 7, 3), (257, 129, 1000)])
def test_gemm_matches_bf16_reference(ta, tb, M_, N_, K_):
    rng = np.random.default_rng(M_ + N_ + K_)
    A = rng.normal(size=(K_, M_) if ta else (M_, K_)).astype(np.float32)
    B = rng.normal(size=(N_, K_) if tb else (K_, N_)).astype(np.float32)
    C = _gb().gemm_test(A, B, M_, N_, K_, ta, tb)
    Ar = M.bf16(A).T if ta else M.bf16(A)
    Br = M.bf16(B).T if tb else M.bf16(B)
    ref = Ar @ Br
    scale = np.sqrt((Ar ** 2).sum(1))[:, None] * np.sqrt((Br ** 2).sum(0))[None, :]
    # products of BF16 values are exact in FP32; what remains is FP32
    # accumulation, far below the BF16 input rounding a wrong cast would show
    assert np.all(np.abs(C - ref) <= 2e-5 * scale + 1e-30)


# widths that are multiples of 8 take the LDS-staged BF16 epilogue, width 60
# the element-wise one; 17,000 rows of width 512 fill the GPU with 128-row
# tiles and end on a ragged tile (17,000 = 132 x 128 + 104)
@pytest.mark.parametrize("dims,rows", [([53, 64, 64, 24], 300), ([843, 512, 512, 512, 336], 512),
                                       ([53, 60, 60, 24], 300), ([200, 512, 512, 24], 17000)])
def test_network_forward_loss_and_gradient_match_reference(dims, rows):
    gb = _gb()
    net = gb.MLP(dims[0], dims[1], len(dims) - 2, dims[-1], seed=1)
    p = M.init_params(dims, seed=4).astype(np.float32)
    net.set_params(p)
    rng = np.random.default_rng(7)
    X = rng.normal(size=(rows, dims[0])).astype(np.float32)
    T = rng.normal(size=(rows, dims[-1])).astype(np.float32)
    Y = net.forward(X)
    yref, _ = M.forward(p, dims, X)
    # The GPU rounds FP32 sums to BF16 where the reference rounds FP64 sums:
    # an activation within the FP32 error of a BF16 rounding boundary rounds
    # the other way (one BF16 step, 2^-8 relative) and moves that row's
    # outputs by about that much times the weights that follow.  Such flips
    # are rare, so the error is small in norm; no element moves by more
    # than a few BF16 steps of the output scale.
    assert np.linalg.norm(Y - yref) <= 1e-3 * np.linalg.norm(yref)
    assert np.abs(Y - yref).max() <= 2 ** -5 * np.abs(yref).max()
    loss, g = net.loss_grad(X, T)
    lref, gref = M.loss_grad(p, dims, X, T)
    assert abs(loss - lref) <= 1e-4 * lref
    assert np.linalg.norm(g - gref) <= 1e-3 * np.linalg.norm(gref)


def test_scaling_statistics_match_reference():
    gb = _gb()
    rng = np.random.default_rng(3)
    X = (rng.normal(size=(5000, 53)) * rng.uniform(0.1, 30, 53) + rng.uniform(-50, 50, 53)).astype(np.float32)
    X[:, 7] = 2.5                                   # a constant column
    T = (rng.normal(size=(5000, 24)) * 3 + 1).astype(np.float32)
    net = gb.MLP(53, 64, 2, 24, seed=1)
    net.fit_scaling(X, T)
    got = net.get_scaling()
    ref = M.scaling(X, T)
    for g, r in zip(got, ref):
        np.testing.assert_allclose(g, r, rtol=2e-6, atol=1e-6)


@pytest.mark.parametrize("dims,rows", [([53, 64, 64, 24], 300), ([843, 512, 512, 512, 336], 512)])
def test_scaled_network_matches_reference(dims, rows):
    gb = _gb()
    net = gb.MLP(dims[0], dims[1], len(dims) - 2, dims[-1], seed=1)
    p = M.init_params(dims, seed=4).astype(np.float32)
    net.set_params(p)
    rng = np.random.default_rng(9)
    X = (rng.normal(size=(rows, dims[0])) * 20 + 5).astype(np.float32)
    T = (rng.normal(size=(rows, dims[-1])) * 0.3 - 2).astype(np.float32)
    net.fit_scaling(X, T)
    sc = net.get_scaling()
    Y = net.forward(X)
    yref, _ = M.forward(p, dims, X, sc=sc)
    assert np.linalg.norm(Y - yref) <= 1e-3 * np.linalg.norm(yref)
    loss, g = net.loss_grad(X, T)
    lref, gref = M.loss_grad(p, dims, X, T, sc=sc)
    assert abs(loss - lref) <= 1e-4 * lref
    assert np.linalg.norm(g - gref) <= 1e-3 * np.linalg.norm(gref)


def test_adam_reduces_the_loss():
    gb = _gb()
    dims = [53, 64, 64, 24]
    net = gb.MLP(dims[0], 64, 2, dims[-1], seed=3)
    rng = np.random.default_rng(0)
    X = rng.normal(size=(512, 53)).astype(np.float32)
    W = rng.normal(size=(53, 24)) / 8
    T = np.tanh(X @ W).astype(np.float32)
    l0 = net.loss_grad(X, T)[0]
    for _ in range(200):
        net.adam_step(X, T, 3e-3)
    assert net.loss_grad(X, T)[0] < 0.1 * l0


def _plan(case, **kw):
    gb = _gb()
    return gb.Plan(case, gb.options(**kw), stream=gb.current_stream())


@pytest.mark.parametrize("n_hvdc", [0, 2])
def test_features_and_targets_match_oracle(n_hvdc):
    import torch
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=2, seed=7, n_hvdc=n_hvdc)
    eta = cases.jitter(cs.eta_min(), 4, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    with _plan(cs) as p:
        p.solve(eta, [0, 1])
        rows, T = p.nn_rows([0, 1])
        X = torch.empty((rows, 5 * T + 3), dtype=torch.float32, device="cuda")
        Y = torch.empty((rows, 2 * T), dtype=torch.float32, device="cuda")
        p.features(eta, [0, 1], X)
        p.targets([0, 1], Y)
        sols = [p.solution(s) for s in (0, 1)]
    X, Y = X.cpu().numpy(), Y.cpu().numpy()
    N = cs.networks[0].n_nodes
    for s in (0, 1):
        Xr = M.features(cs, s, eta)
        np.testing.assert_allclose(X[s * N:(s + 1) * N], Xr, rtol=1e-5, atol=1e-5)
        qp = D.assemble(cs, s, eta)
        Yr = M.targets(qp, sols[s][0].astype(np.float64), sols[s][1])
        np.testing.assert_allclose(Y[s * N:(s + 1) * N], Yr, rtol=1e-5, atol=1e-6)


def test_features_of_several_networks_match_oracle():
    """Scenarios on different networks (each its own capacity slice of eta)."""
    import torch
    cs = cases.config2(S=12)
    byT = {}
    for s, sc in enumerate(cs.scenarios):
        byT.setdefault(sc.T, []).append(s)
    scen = max(byT.values(), key=len)[:3]
    eta = cases.jitter(cs.eta_min(), 5, amount=0.2, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    off = cs.eta_offsets()
    with _plan(cs) as p:
        rows, T = p.nn_rows(scen)
        X = torch.empty((rows, 5 * T + 3), dtype=torch.float32, device="cuda")
        p.features(eta, scen, X)
    X = X.cpu().numpy()
    r = 0
    for s in scen:
        n = cs.scenarios[s].network
        Xr = M.features(cs, s, eta[off[n]:off[n + 1]])
        np.testing.assert_allclose(X[r:r + Xr.shape[0]], Xr, rtol=1e-5, atol=1e-5)
        r += Xr.shape[0]
    assert r == rows


def test_seeding_from_exact_prices_and_angles_saves_iterations():
    """A perfect prediction (the oracle's own prices and angles) seeds a start
    that is accepted and converges, over four scenarios, in well under the
    cold-start iterations (the batteries and the marginal generators are
    still left to the solver)."""
    import torch
    cs = cases.small_geo(n_nodes=40, G=120, B=10, T=24, S=4, seed=11)
    scen = [0, 1, 2, 3]
    eta = cases.jitter(cs.eta_min(), 3, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    P, objs = [], []
    for s in scen:
        qp = D.assemble(cs, s, eta)
        sol = D.solve(qp)
        P.append(M.targets(qp, sol.x, sol.y))
        objs.append(sol.obj)
    P = torch.tensor(np.concatenate(P), dtype=torch.float32, device="cuda")
    with _plan(cs, block=256, variant=1, check_every=64) as p:
        _, s_cold, _ = p.solve(eta, scen, warm=0)
        p.start_from_prediction(eta, scen, P)
        c_seed, s_seed, rc = p.solve(eta, scen, warm=1)
    assert rc == 0
    assert all(st["start"] == 1 for st in s_seed)
    np.testing.assert_allclose(c_seed, objs, rtol=1e-4)
    n_seed, n_cold = sum(st["iters"] for st in s_seed), sum(st["iters"] for st in s_cold)
    print(f"\n[gpu] seeded {[st['iters'] for st in s_seed]} cold {[st['iters'] for st in s_cold]}", flush=True)
    assert n_seed <= 0.6 * n_cold, (n_seed, n_cold)


def test_stalled_warm_start_restarts_exactly_as_a_cold_start():
    """With the stall limit forced down to 1 % of the cold iterations, a warm
    start from the solution at other capacities is abandoned at its first
    check and the scenario then runs exactly as a cold solve does."""
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=2, seed=7)
    eta = cases.jitter(cs.eta_min(), 4, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    eta2 = cases.jitter(cs.eta_min(), 5, amount=5.0, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    kw = dict(block=256, variant=1, check_every=64)
    with _plan(cs, **kw) as ref:
        c_ref, s_ref, _ = ref.solve(eta2, [0, 1], warm=0)
    with _plan(cs, stall_pct=1, **kw) as p:
        p.solve(eta, [0, 1], warm=0)
        c, st, rc = p.solve(eta2, [0, 1], warm=1)
    assert rc == 0
    assert [x["start"] for x in st] == [3, 3]
    np.testing.assert_array_equal(c, c_ref)
    assert [x["iters"] for x in st] == [64 + x["iters"] for x in s_ref]


def test_bad_prediction_is_rejected_and_the_solve_matches_cold():
    """A prediction far from any solution (node prices of +-2e10 at random)
    scores far below zero on the exact dual function: every scenario starts
    cold (stats start = 2) and the solve is the cold solve, bit for bit."""
    import torch
    cs = cases.small_geo(n_nodes=12, G=30, B=3, T=24, S=2, seed=7)
    eta = cases.jitter(cs.eta_min(), 4, eta_min=cs.eta_min(), eta_max=cs.eta_max())
    with _plan(cs, block=256, variant=1, check_every=64) as p:
        c0, s0, _ = p.solve(eta, [0, 1], warm=0)
        assert all(st["start"] == 0 for st in s0)
        c1, s1, _ = p.solve(eta, [0, 1], warm=1)      # previous solution: accepted
        assert all(st["start"] == 1 for st in s1)
        assert max(st["iters"] for st in s1) < max(st["iters"] for st in s0)
        rows, T = p.nn_rows([0, 1])
        g = torch.Generator(device="cuda")
        g.manual_seed(0)
        P = 20.0 * torch.sign(torch.randn((rows, 2 * T), device="cuda", generator=g))
        p.start_from_prediction(eta, [0, 1], P)
        c2, s2, _ = p.solve(eta, [0, 1], warm=1)
    assert all(st["start"] == 2 for st in s2)
    assert [st["iters"] for st in s2] == [st["iters"] for st in s0]
    np.testing.assert_array_equal(c2, c0)


def test_trained_network_seeds_held_out_solves():
    """Collect solutions along short planning runs under four storage costs,
    train on them, then on a held-out run (a fifth cost) compare seeded solves
    with cold solves and with a network of random weights (the ablation).
    Every seeded solve reaches the cold optimum; the trained network saves
    iterations over both."""
    import time
    import torch
    from paper_2410_13055_amd.warmstart import LearnedWarmStart
    cs = cases.small_geo(n_nodes=40, G=120, B=10, T=24, S=4, seed=11)
    net0 = cs.networks[0]
    G, L = net0.n_gens, net0.n_lines
    scen = [0, 1, 2, 3]
    with _plan(cs) as p:
        ws = LearnedWarmStart(p, cs.scenarios[0].T, seed=0)

        def run(price, steps, collect):
            gamma = cs.gamma().copy()
            gamma[G + L:] = cases.storage_gamma_per_mw(price)
            eta = cs.eta_min().copy()
            p.solve(eta, scen)
            g0, _, _ = p.grad(scen)
            alpha = 0.05 * (cs.eta_max() - cs.eta_min()).min() / np.abs(gamma + g0).max()
            pts = []
            for k in range(steps):
                eta_new, phi, delta, rc = p.step(alpha, scen, gamma, eta, warm=1 if k else 0)
                if collect:
                    ws.collect(eta, scen)
                pts.append(eta.copy())
                eta = eta_new
            return pts

        for price in (100.0, 175.0, 325.0, 400.0):
            run(price, 5, True)
        losses = ws.train(epochs=260, batch_rows=1024, lr=1e-3)
        assert losses[-1] < 0.5 * losses[0], (losses[0], losses[-1])
        held = run(250.0, 4, False)
        rnd = LearnedWarmStart(p, cs.scenarios[0].T, seed=99)   # untrained ablation
        it_cold, it_warm, it_rand, t_cold, t_warm = [], [], [], 0.0, 0.0
        for eta in held:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cc, st, _ = p.solve(eta, scen, warm=0)
            t_cold += time.perf_counter() - t0
            it_cold.append(max(s["iters"] for s in st))
            cw, st, dt = ws.solve(eta, scen)
            t_warm += dt
            it_warm.append(max(s["iters"] for s in st))
            assert all(s["status"] == 0 for s in st)
            np.testing.assert_allclose(cw, cc, rtol=2e-4)
            _, st, _ = rnd.solve(eta, scen)
            it_rand.append(max(s["iters"] for s in st))
            assert all(s["status"] == 0 for s in st)
    print(f"\n[gpu] cold iters {it_cold} {t_cold:.3f}s | learned {it_warm} {t_warm:.3f}s | random {it_rand}",
          flush=True)
    assert sum(it_warm) <= 0.8 * sum(it_cold)
    assert sum(it_warm) < sum(it_rand)
