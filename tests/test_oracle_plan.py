"""Pins for the planning layer of the oracle (Section 2.1 eq. (1) and the
projected step of Section 2.2): with h = c the bilevel objective must agree
with the classical joint convex QP over (eta, x), whose optimum is a lower
bound that projected gradient descent approaches."""
import numpy as np

from paper_2410_13055_amd import cases
from oracle import plan as P


def test_joint_qp_pins_bilevel_objective_and_descent():
    cs = cases.config0()
    eta_s, val, status = P.joint_optimum(cs)
    assert status == "optimal"
    f_star, _ = P.phi(cs, eta_s, [0], 0.0)
    # the dispatch map evaluated at the joint optimum reproduces its value
    assert abs(f_star - val) <= 1e-9 * abs(val)
    eta = cs.eta_min().copy()
    f0, d0 = P.phi(cs, eta, [0], 0.0)
    alpha = 0.1 * (cs.eta_max() - cs.eta_min()).min() / np.abs(d0).max()
    best = f0
    for k in range(40):
        eta, f, d = P.projected_step(cs, eta, alpha / np.sqrt(1 + k / 10), [0], 0.0)
        assert f >= val - 1e-9 * abs(val)          # joint optimum is a lower bound
        assert np.all(eta >= cs.eta_min()) and np.all(eta <= cs.eta_max())
        best = min(best, f)
    assert (best - val) <= 0.05 * (f0 - val)
