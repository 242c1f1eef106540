"""Learned warm start of the dispatch solver.

A small MLP maps per-node features (own and neighbouring load and available
capacity profiles, local capacities) to that node's price and angle
profiles; the prediction seeds the solver (``Plan.start_from_prediction``),
which then runs to the usual KKT tolerance, so a poor prediction costs
iterations but never accuracy.  Training data are the solver's own solutions
collected along planning runs.  Feature extraction, the network's forward
and backward passes, Adam and the seeding all run in the library; torch
only holds the device matrices.
"""
from __future__ import annotations

import time

import numpy as np

from . import gridplan


class LearnedWarmStart:
    def __init__(self, plan: gridplan.Plan, T: int, width: int = 512, hidden_layers: int = 3, seed: int = 0):
        import torch
        self.torch = torch
        self.plan = plan
        self.T = T
        self.n_in, self.n_out = 5 * T + 3, 2 * T
        self.net = gridplan.MLP(self.n_in, width, hidden_layers, self.n_out, seed=seed,
                                stream=gridplan.current_stream())
        self.X, self.Y = [], []
        self.history = []
        self.scaled = False

    @property
    def rows(self):
        return sum(x.shape[0] for x in self.X)

    def _alloc(self, rows, cols):
        return self.torch.empty((rows, cols), dtype=self.torch.float32, device="cuda")

    def features(self, eta, scen):
        rows, T = self.plan.nn_rows(scen)
        assert T == self.T
        X = self._alloc(rows, self.n_in)
        self.plan.features(eta, scen, X)
        return X

    def collect(self, eta, scen):
        """Record (features, solution) rows of the scenarios' stored solutions,
        which must have been solved at eta."""
        rows, _ = self.plan.nn_rows(scen)
        X = self.features(eta, scen)
        Y = self._alloc(rows, self.n_out)
        self.plan.targets(scen, Y)
        self.X.append(X)
        self.Y.append(Y)

    def train(self, epochs: int = 20, batch_rows: int = 4096, lr: float = 1e-3, seed: int = 0):
        """Adam on the mean squared error over the collected rows, inputs and
        targets standardised by the statistics of the data at the first
        call; minibatches are contiguous row ranges visited in a shuffled
        order.  Returns the mean loss per epoch (standardised units)."""
        torch = self.torch
        X = torch.cat(self.X) if len(self.X) > 1 else self.X[0]
        Y = torch.cat(self.Y) if len(self.Y) > 1 else self.Y[0]
        if not self.scaled:
            self.net.fit_scaling(X, Y)
            self.scaled = True
        n = X.shape[0]
        starts = np.arange(0, n, batch_rows)
        rng = np.random.default_rng(seed)
        losses = []
        for ep in range(epochs):
            tot = 0.0
            for i in rng.permutation(starts):
                j = min(i + batch_rows, n)
                tot += self.net.adam_step(X[i:j], Y[i:j], lr) * (j - i)
            losses.append(tot / n)
        self.history += losses
        return losses

    def loss(self, X, Y):
        return self.net.loss_grad(X, Y)[0]

    def seed(self, eta, scen):
        """Predict and seed the scenarios' next warm solve."""
        X = self.features(eta, scen)
        P = self.net.forward(X)
        self.plan.start_from_prediction(eta, scen, P)
        return P

    def solve(self, eta, scen):
        """Seeded solve; returns (cost, stats, seconds including inference)."""
        self.torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.seed(eta, scen)
        cost, st, rc = self.plan.solve(eta, scen, warm=1)
        self.torch.cuda.synchronize()
        return cost, st, time.perf_counter() - t0
