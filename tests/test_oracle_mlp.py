"""Pins for the warm-start network reference: the BF16 rounding matches a
library implementation (torch's bfloat16 cast), and the unrounded network's
gradient matches central finite differences."""
import numpy as np
import torch

from oracle import mlp as M


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e4, 500), rng.normal(0, 1e-5, 500),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0, 3.0e38]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x), ref)


def test_unrounded_gradient_matches_central_differences():
    dims = [7, 9, 9, 4]
    p = M.init_params(dims, seed=3)
    rng = np.random.default_rng(1)
    X = rng.normal(size=(11, 7))
    T = rng.normal(size=(11, 4))
    loss, g = M.loss_grad(p, dims, X, T, rounding=False)
    h = 1e-6
    idx = rng.choice(p.size, 40, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = M.loss_grad(p + e, dims, X, T, rounding=False)
        lm, _ = M.loss_grad(p - e, dims, X, T, rounding=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_rounded_network_is_close_to_unrounded():
    dims = [16, 32, 8]
    p = M.init_params(dims, seed=5)
    X = np.random.default_rng(2).normal(size=(20, 16))
    y0, _ = M.forward(p, dims, X, rounding=False)
    y1, _ = M.forward(p, dims, X, rounding=True)
    # bf16 keeps 8 significant bits: relative error of a layer ~ 2^-8
    assert np.abs(y1 - y0).max() <= 3e-2 * np.abs(y0).max()


def test_features_shape_and_physical_sums():
    from paper_2410_13055_amd import cases
    cs = cases.config0()
    eta = cs.eta_min()
    X = M.features(cs, 0, eta)
    T = cs.scenarios[0].T
    assert X.shape == (cs.networks[0].n_nodes, 5 * T + 3)
    # node loads sum to the system load; available capacity sums to the fleet's
    np.testing.assert_allclose(X[:, :T].sum(0) * 100, cs.scenarios[0].load.sum(0))
    G = cs.networks[0].n_gens
    avail = (cs.scenarios[0].avail * eta[:G, None]).sum(0)
    np.testing.assert_allclose((X[:, T:2 * T] + X[:, 2 * T:3 * T]).sum(0) * 100, avail)


def test_colstats_closed_forms():
    a, b = 3.5, -1.25
    A = np.zeros((10, 3))
    A[0::2, 0], A[1::2, 0] = a, b          # two values, equal counts
    A[:, 1] = 7.0                          # no spread: centred only
    A[:, 2] = np.arange(10)                # 0..9: mean 4.5, variance 8.25
    mu, sd = M.colstats(A)
    np.testing.assert_allclose(mu, [(a + b) / 2, 7.0, 4.5], rtol=1e-7)
    np.testing.assert_allclose(sd, [abs(a - b) / 2, 1.0, np.sqrt(8.25)], rtol=1e-7)


def test_scaled_gradient_matches_central_differences():
    dims = [6, 8, 3]
    p = M.init_params(dims, seed=7)
    rng = np.random.default_rng(4)
    X = rng.normal(3.0, 5.0, size=(13, 6))
    T = rng.normal(-2.0, 0.1, size=(13, 3))
    sc = M.scaling(X, T)
    loss, g = M.loss_grad(p, dims, X, T, rounding=False, sc=sc)
    h = 1e-6
    for i in rng.choice(p.size, 30, replace=False):
        e = np.zeros_like(p)
        e[i] = h
        fd = (M.loss_grad(p + e, dims, X, T, False, sc)[0] - M.loss_grad(p - e, dims, X, T, False, sc)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_scaling_is_equivariant_to_affine_target_changes():
    """Targets a*T + b (per column, a > 0) give the same standardised
    problem: the same loss, and predictions a*y + b."""
    dims = [5, 16, 4]
    p = M.init_params(dims, seed=8)
    rng = np.random.default_rng(6)
    X = rng.normal(size=(40, 5)).astype(np.float32)
    T = rng.normal(size=(40, 4)).astype(np.float32)
    a = np.array([2.0, 0.5, 4.0, 1.0], np.float32)
    b = np.array([1.0, -3.0, 0.0, 8.0], np.float32)
    T2 = T * a + b
    sc1, sc2 = M.scaling(X, T), M.scaling(X, T2)
    l1, _ = M.loss_grad(p, dims, X, T, rounding=False, sc=sc1)
    l2, _ = M.loss_grad(p, dims, X, T2, rounding=False, sc=sc2)
    assert abs(l1 - l2) <= 1e-5 * l1
    y1, _ = M.forward(p, dims, X, rounding=False, sc=sc1)
    y2, _ = M.forward(p, dims, X, rounding=False, sc=sc2)
    np.testing.assert_allclose(y2, y1 * a + b, rtol=1e-5, atol=1e-5)
