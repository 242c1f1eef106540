"""FP64 reference for the learned warm start.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The warm-start network is not part of the paper (its warm start reuses a
previous plan, Section 2.2 "Interactivity"); this module states what the GPU
network and its feature extraction compute, in plain numpy:

* ``bf16``: round-to-nearest-even of an FP32 value to bfloat16 (8 exponent
  bits, 7 stored mantissa bits), returned as FP64.
* ``forward`` / ``loss_grad``: an MLP x -> relu(x W_0 + b_0) -> ... -> y with
  the GPU's cast points: every GEMM operand (input, activations, weights,
  output gradients) rounded to BF16, products accumulated exactly (FP64),
  biases and the loss in full precision.  ``rounding=False`` gives the
  unrounded FP64 network used for the finite-difference pin.
* ``colstats`` and ``scaling``: optional standardisation of inputs and
  targets by column mean and standard deviation.  The network then sees
  (x - mu_x)/sd_x (FP32 arithmetic, then BF16), is trained on
  (y - mu_y)/sd_y (the loss is in those units) and ``forward`` returns
  predictions in target units.
* ``features`` / ``targets``: the per-node inputs and outputs of the network
  for one scenario (same definitions as the library's documentation).
"""
from __future__ import annotations

import numpy as np

from . import dispatch as D


def bf16(x):
    """Round FP32 values (given as any float array) to bfloat16, nearest-even."""
    a = np.asarray(x, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(a)
    out[nan] = np.nan
    return out


def unpack(params, dims):
    """Flat parameters (all weights [in x out] in layer order, then biases)."""
    W, B, o = [], [], 0
    for i in range(len(dims) - 1):
        n = dims[i] * dims[i + 1]
        W.append(np.asarray(params[o:o + n], np.float64).reshape(dims[i], dims[i + 1]))
        o += n
    for i in range(len(dims) - 1):
        B.append(np.asarray(params[o:o + dims[i + 1]], np.float64))
        o += dims[i + 1]
    return W, B


def colstats(A):
    """Column mean and population standard deviation of A, as FP32; a column
    whose spread is below 1e-6 (1 + |mean|) keeps sd = 1 (it is only
    centred)."""
    A = np.asarray(A, np.float64)
    mu = A.mean(axis=0)
    sd = np.sqrt(np.maximum((A * A).mean(axis=0) - mu * mu, 0.0))
    sd = np.where(sd > 1e-6 * (1.0 + np.abs(mu)), sd, 1.0)
    return mu.astype(np.float32), sd.astype(np.float32)


def scaling(X, T):
    """(x_mu, x_sd, y_mu, y_sd) of a training set."""
    return (*colstats(X), *colstats(T))


def _standardise(A, mu, sd):
    """(A - mu) * (1/sd) in FP32 arithmetic."""
    A = np.asarray(A, np.float32)
    return ((A - np.float32(1) * mu) * (np.float32(1) / sd)).astype(np.float32).astype(np.float64)


def _net(params, dims, X, rounding, sc):
    r = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    W, B = unpack(params, dims)
    h = r(_standardise(X, sc[0], sc[1]) if sc is not None else X)
    acts = [h]
    L = len(W)
    for l in range(L):
        z = h @ r(W[l]) + B[l]
        if l + 1 < L:
            h = r(np.maximum(z, 0.0))
            acts.append(h)
        else:
            y = np.asarray(z, np.float32).astype(np.float64) if rounding else z
    return y, acts


def forward(params, dims, X, rounding=True, sc=None):
    """Network output in target units (and the BF16 activations)."""
    z, acts = _net(params, dims, X, rounding, sc)
    if sc is not None:
        z = (np.asarray(z, np.float32) * sc[3] + sc[2]).astype(np.float32).astype(np.float64)
    return z, acts


def loss_grad(params, dims, X, T, rounding=True, sc=None):
    """Mean squared error over every output and its gradient (flat); with a
    scaling, in standardised target units."""
    r = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    W, B = unpack(params, dims)
    y, acts = _net(params, dims, X, rounding, sc)
    T = _standardise(T, sc[2], sc[3]) if sc is not None else np.asarray(T, np.float64)
    n = y.size
    d = y - T
    loss = float(np.sum(d * d) / n)
    g = 2.0 * d / n
    dW, dB = [None] * len(W), [None] * len(W)
    gb = r(g)
    for l in range(len(W) - 1, -1, -1):
        dW[l] = acts[l].T @ gb
        dB[l] = g.sum(axis=0)
        if l > 0:
            g = (gb @ r(W[l]).T) * (acts[l] > 0)
            gb = r(g)
    flat = np.concatenate([w.ravel() for w in dW] + [b for b in dB])
    return loss, flat


def init_params(dims, seed=0):
    rng = np.random.default_rng(seed)
    ws, bs = [], []
    for i in range(len(dims) - 1):
        a = np.sqrt(6.0 / dims[i])
        ws.append(rng.uniform(-a, a, size=(dims[i], dims[i + 1])).ravel())
        bs.append(rng.uniform(-0.1, 0.1, size=dims[i + 1]))
    return np.concatenate(ws + bs)


def features(case, s, eta_net):
    """Node features of scenario s at the network capacities eta_net:
    rows = nodes, columns = [load | renewable available capacity | thermal
    available capacity | neighbours' load | neighbours' renewable available
    capacity] (each T hours, MW/100) then [battery capacity, incident line
    capacity, thermal nameplate] (MW/100).  Renewable means zero cost."""
    sc = case.scenarios[s]
    net = case.networks[sc.network]
    N, T, G, L = net.n_nodes, sc.T, net.n_gens, net.n_lines
    eg, el, eb = eta_net[:G], eta_net[G:G + L], eta_net[G + L:]
    cap = sc.avail * eg[:, None]
    ren = np.zeros((N, T))
    thr = np.zeros((N, T))
    for g in range(G):
        (thr if net.gen_cost[g] > 0 else ren)[net.gen_node[g]] += cap[g]
    nl = np.zeros((N, T))
    nren = np.zeros((N, T))
    lcap = np.zeros(N)
    for l in range(L):
        a, b = net.line_from[l], net.line_to[l]
        nl[a] += sc.load[b]
        nl[b] += sc.load[a]
        nren[a] += ren[b]
        nren[b] += ren[a]
        lcap[a] += el[l]
        lcap[b] += el[l]
    bcap = np.zeros(N)
    for k in range(net.n_batt):
        bcap[net.batt_node[k]] += eb[k]
    gcap = np.zeros(N)
    for g in range(G):
        if net.gen_cost[g] > 0:
            gcap[net.gen_node[g]] += eg[g]
    X = np.concatenate([sc.load, ren, thr, nl, nren, bcap[:, None], lcap[:, None], gcap[:, None]], axis=1)
    return X / 100.0


def targets(qp: D.QP, x, y):
    """Network outputs of a solved scenario: asinh(price/100), angle/10."""
    N, T = qp.dims["N"], qp.dims["T"]
    pi = np.asarray(y)[qp.dims["rs"]["bal"]].reshape(N, T)
    th = np.asarray(x)[qp.dims["vs"]["th"]].reshape(N, T)
    return np.concatenate([np.arcsinh(pi / 100.0), th / 10.0], axis=1)
