"""The byte models behind the bench line's roofline, counted by hand.

Method bytes of one ADMM iteration: every FP32 primal read and written
(8 B per variable), every FP32 dual read and written (8 B per equality
row), every time-varying FP32 parameter read once (4 B per generator-hour
of availability and per node-hour of load)."""
import numpy as np

import bench
from paper_2410_13055_amd import cases


def test_method_bytes_of_the_1000_node_workload():
    # per scenario: variables (5000 + 1500 + 2*1000 + 3*500) * 168 =
    # 1,680,000; rows (1000 + 1500 + 500) * 168 = 504,000; parameters
    # (5000 + 1000) * 168 = 1,008,000 -> 21,504,000 B; 16 scenarios
    case = cases.config4(S=16)
    assert bench.method_bytes(case, range(16)) == 16 * (8 * 1_680_000 + 8 * 504_000 + 4 * 1_008_000)
    assert bench.method_bytes(case, range(16)) == 344_064_000


def test_design_bytes_of_the_1000_node_workload():
    # variable sweep: 12 B per variable, 12 B per row, 4 B per
    # generator-hour; row sweep: 4 B per variable, 8 B per row, 4 B per
    # node-hour
    case = cases.config4(S=16)
    ab = bench.algorithmic_bytes(case, range(16))
    nx, ny, gt, nt = 1_680_000 * 16, 504_000 * 16, 840_000 * 16, 168_000 * 16
    assert (ab["n_x"], ab["n_y"]) == (nx, ny)
    assert ab["primal"] == 12 * nx + 12 * ny + 4 * gt == 473_088_000
    assert ab["dual"] == 4 * nx + 8 * ny + 4 * nt == 182_784_000


def test_links_and_ramps_in_the_counts():
    # an HVDC link has a flow variable and no flow row; a ramp-limited
    # unit adds one variable and one row per hour
    cs = cases.small_geo(n_nodes=8, G=16, B=2, T=24, S=1, seed=40, n_hvdc=1, gas_ramp=0.12)
    n = cs.networks[0]
    R = int((n.gen_ramp > 0).sum())
    assert R > 0 and n.n_hvdc == 1
    nx = (n.n_gens + n.n_lines + 2 * n.n_nodes + 3 * n.n_batt + R) * 24
    ny = (n.n_nodes + (n.n_lines - 1) + n.n_batt + R) * 24
    assert bench.method_bytes(cs, [0]) == 8 * nx + 8 * ny + 4 * (n.n_gens + n.n_nodes) * 24
    # the oracle's QP of the same scenario has exactly these dimensions
    from oracle import dispatch as D
    qp = D.assemble(cs, 0, cs.eta_min())
    assert (qp.n, qp.m) == (nx, ny)
