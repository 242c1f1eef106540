"""Seeded synthetic grids for the expansion-planning dispatch problems.

This module only draws *inputs*: network topology, device parameters, capacity
boxes, investment costs and per-scenario hourly profiles.  It holds none of the
dispatch method's arithmetic (no constraint assembly, no bounds from
capacities, no solver), so both the CPU oracle and the GPU path can consume it.

The paper's experiments use the PyPSA-USA Western Interconnect (Section 3,
"Results", data paragraph); that dataset is not available here, so these
generators stand in for it with the same kind of structure: a meshed
transmission network, thermal/solar/wind generators placed at nodes,
4-hour batteries, hourly loads with a daily cycle, and independent scenarios
(Section 3 treats each day as an independent scenario).

Every floating value that the GPU consumes in FP32 is rounded to an FP32
representable number here, so the oracle (FP64) and the GPU path solve exactly
the same problem.

Capacity vector layout (per network): ``eta = [generators | lines | batteries]``
(the paper's eta in R^K, Section 2.1).  Across networks the vectors are
concatenated in network order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

GAS, SOLAR, WIND = 0, 1, 2

#: constants shared by every configuration
REG_R = 1e-3          # quadratic regulariser, $/MW^2 h
LAMBDA_U = 1e4        # unserved-load penalty, $/MWh
EFF = 0.95            # battery charging efficiency (one-way, on charge)
HOURS = 4.0           # battery duration, h (SOC capacity = HOURS * power capacity)
GAS_EMIS = 0.4        # t CO2 / MWh for gas units


def _f32(a):
    """Round to FP32-representable values, returned as float64."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@dataclasses.dataclass
class Network:
    n_nodes: int
    line_from: np.ndarray   # int32 [L]
    line_to: np.ndarray     # int32 [L]
    line_beta: np.ndarray   # float64 [L] susceptance (MW per rad)
    gen_node: np.ndarray    # int32 [G]
    gen_kind: np.ndarray    # int32 [G] GAS / SOLAR / WIND
    gen_cost: np.ndarray    # float64 [G] $/MWh
    gen_emis: np.ndarray    # float64 [G] t/MWh
    batt_node: np.ndarray   # int32 [B]
    eta_min: np.ndarray     # float64 [K]
    eta_max: np.ndarray     # float64 [K]
    gamma: np.ndarray       # float64 [K] $/MW-yr investment cost
    n_hvdc: int = 0         # the last n_hvdc lines are HVDC links (their beta is unused)
    beta_scales: bool = False  # AC susceptance beta_l * eta_l / eta_min_l (parallel circuits)
    gen_ramp: Optional[np.ndarray] = None  # float64 [G]: share of capacity a unit can move per hour (0: no limit)

    @property
    def n_lines(self) -> int:
        return int(self.line_from.shape[0])

    @property
    def n_ac(self) -> int:
        return self.n_lines - int(self.n_hvdc)

    @property
    def n_gens(self) -> int:
        return int(self.gen_node.shape[0])

    @property
    def n_batt(self) -> int:
        return int(self.batt_node.shape[0])

    @property
    def K(self) -> int:
        return self.n_gens + self.n_lines + self.n_batt


@dataclasses.dataclass
class Scenario:
    network: int
    T: int
    avail: np.ndarray   # float64 (FP32 values) [G, T], availability factor in [0, 1]
    load: np.ndarray    # float64 (FP32 values) [N, T], MW
    weight: float       # annualisation weight 8760 / T


@dataclasses.dataclass
class Case:
    name: str
    networks: List[Network]
    scenarios: List[Scenario]
    r: float = REG_R
    lambda_u: float = LAMBDA_U
    eff: float = EFF
    hours: float = HOURS
    omega: float = 0.0      # carbon weight, $/t (planner objective only)

    @property
    def K(self) -> int:
        return sum(n.K for n in self.networks)

    def eta_offsets(self) -> np.ndarray:
        off = np.zeros(len(self.networks) + 1, dtype=np.int64)
        for i, n in enumerate(self.networks):
            off[i + 1] = off[i] + n.K
        return off

    def eta_min(self) -> np.ndarray:
        return np.concatenate([n.eta_min for n in self.networks])

    def eta_max(self) -> np.ndarray:
        return np.concatenate([n.eta_max for n in self.networks])

    def gamma(self) -> np.ndarray:
        return np.concatenate([n.gamma for n in self.networks])

    def scenario_hours(self, idx=None) -> int:
        idx = range(len(self.scenarios)) if idx is None else idx
        return int(sum(self.scenarios[i].T for i in idx))


# --------------------------------------------------------------------------
# topology
# --------------------------------------------------------------------------

def ring_with_chords(n: int = 6, chords=((0, 3), (2, 5))):
    """Ring of ``n`` nodes plus chords (the tiny case)."""
    edges = [(i, (i + 1) % n) for i in range(n)] + list(chords)
    a = np.array([min(e) for e in edges], dtype=np.int32)
    b = np.array([max(e) for e in edges], dtype=np.int32)
    return a, b


def geometric_mst_plus(rng: np.random.Generator, n: int, n_lines: int):
    """Points uniform in the unit square; Euclidean MST (n-1 edges) plus the
    shortest remaining pairs until exactly ``n_lines`` edges.  Connected by
    construction; mean degree 2*n_lines/n."""
    from scipy.sparse.csgraph import minimum_spanning_tree

    pts = rng.random((n, 2))
    d = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1))
    mst = minimum_spanning_tree(np.triu(d, 1)).tocoo()
    used = set()
    edges = []
    for i, j in zip(mst.row.tolist(), mst.col.tolist()):
        a, b = min(i, j), max(i, j)
        used.add((a, b))
        edges.append((a, b))
    iu, ju = np.triu_indices(n, 1)
    order = np.argsort(d[iu, ju], kind="stable")
    for k in order:
        if len(edges) >= n_lines:
            break
        a, b = int(iu[k]), int(ju[k])
        if (a, b) in used:
            continue
        used.add((a, b))
        edges.append((a, b))
    e = np.array(edges, dtype=np.int32)
    return e[:, 0].copy(), e[:, 1].copy()


# --------------------------------------------------------------------------
# profiles
# --------------------------------------------------------------------------

def _loads(rng, n_nodes, T):
    scale = 100.0 * rng.lognormal(0.0, 0.2, size=n_nodes)
    t = np.arange(T)
    shape = 1.0 + 0.3 * np.sin(2.0 * math.pi * (t - 12) / 24.0)
    return _f32(scale[:, None] * shape[None, :])


def _avail(rng, kinds, T):
    G = kinds.shape[0]
    t = np.arange(T)
    sun = np.maximum(0.0, np.sin(2.0 * math.pi * t / 24.0 - math.pi / 2.0))
    a = np.ones((G, T))
    sol = kinds == SOLAR
    wnd = kinds == WIND
    a[sol] = sun[None, :] * rng.beta(5.0, 2.0, size=(int(sol.sum()), T))
    a[wnd] = rng.beta(2.0, 5.0, size=(int(wnd.sum()), T))
    return _f32(a)


def _kinds(rng, G, fixed_counts=None):
    if fixed_counts is not None:
        k = np.concatenate([np.full(c, i, dtype=np.int32) for i, c in enumerate(fixed_counts)])
    else:
        n_gas = int(round(0.4 * G))
        n_sol = int(round(0.3 * G))
        n_wnd = G - n_gas - n_sol
        k = np.concatenate([np.full(n_gas, GAS), np.full(n_sol, SOLAR),
                            np.full(n_wnd, WIND)]).astype(np.int32)
    return k


def _network(rng, n_nodes, lf, lt, kinds, B, peak, storage_gamma=None):
    L = lf.shape[0]
    G = kinds.shape[0]
    gen_node = rng.integers(0, n_nodes, size=G).astype(np.int32)
    cost = np.where(kinds == GAS, rng.uniform(30.0, 80.0, size=G), 0.0)
    emis = np.where(kinds == GAS, GAS_EMIS, 0.0)
    beta = rng.uniform(5.0, 20.0, size=L)
    batt_node = rng.integers(0, n_nodes, size=B).astype(np.int32)

    g_min = rng.uniform(0.5, 1.5, size=G) * 1.2 * peak / G
    g_max = g_min + 2.0 * peak / G
    l_min = rng.uniform(50.0, 150.0, size=L)
    l_max = 4.0 * l_min
    b_min = rng.uniform(0.5, 1.5, size=B) * 0.05 * peak / max(B, 1)
    b_max = b_min + 0.2 * peak / max(B, 1)
    eta_min = np.concatenate([g_min, l_min, b_min])
    eta_max = np.concatenate([g_max, l_max, b_max])
    gamma = rng.uniform(50e3, 150e3, size=G + L + B)
    if storage_gamma is not None:
        gamma[G + L:] = storage_gamma
    return Network(
        n_nodes=int(n_nodes), line_from=lf.astype(np.int32), line_to=lt.astype(np.int32),
        line_beta=_f32(beta), gen_node=gen_node, gen_kind=kinds.astype(np.int32),
        gen_cost=_f32(cost), gen_emis=_f32(emis), batt_node=batt_node,
        eta_min=_f32(eta_min), eta_max=_f32(eta_max), gamma=_f32(gamma))


def storage_gamma_per_mw(price_per_kwh: float, hours: float = HOURS,
                         rate: float = 0.07, years: int = 15) -> float:
    """Annualised storage investment cost in $/MW-yr from a capital cost in
    $/kWh of energy: price * 1000 kWh/MWh * hours * CRF(rate, years)."""
    crf = rate * (1 + rate) ** years / ((1 + rate) ** years - 1)
    return price_per_kwh * 1000.0 * hours * crf


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------

def hvdc_links(seed, n_nodes, lf, lt, n_hvdc):
    """``n_hvdc`` HVDC links between distinct node pairs that no AC line
    joins (long-distance links in the paper's 500-node case, Section 3.1),
    drawn from their own stream so the AC part of a case does not change."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 0x4456])))
    used = {(min(a, b), max(a, b)) for a, b in zip(lf.tolist(), lt.tolist())}
    hf, ht = [], []
    while len(hf) < n_hvdc:
        a, b = (int(v) for v in rng.choice(n_nodes, 2, replace=False))
        if (min(a, b), max(a, b)) in used:
            continue
        used.add((min(a, b), max(a, b)))
        hf.append(a)
        ht.append(b)
    return (np.concatenate([lf, np.array(hf, np.int32)]).astype(np.int32),
            np.concatenate([lt, np.array(ht, np.int32)]).astype(np.int32))


def _uniform_case(name, cfg_id, n_nodes, G, B, T, S, topo, omega=0.0,
                  fixed_counts=None, storage_price=None, seed=None, n_hvdc=0):
    ss = np.random.SeedSequence(cfg_id if seed is None else seed)
    net_ss, *scen_ss = ss.spawn(S + 1)
    net_rng = np.random.Generator(np.random.PCG64(net_ss))
    if topo == "ring":
        lf, lt = ring_with_chords(n_nodes)
    else:
        lf, lt = geometric_mst_plus(net_rng, n_nodes, int(round(1.5 * n_nodes)))
    if n_hvdc:
        lf, lt = hvdc_links(cfg_id if seed is None else seed, n_nodes, lf, lt, n_hvdc)
    kinds = _kinds(net_rng, G, fixed_counts)
    scen = []
    loads = []
    for s in range(S):
        rng = np.random.Generator(np.random.PCG64(scen_ss[s]))
        ld = _loads(rng, n_nodes, T)
        av = _avail(rng, kinds, T)
        loads.append(ld)
        scen.append(Scenario(network=0, T=T, avail=av, load=ld, weight=8760.0 / T))
    peak = float(np.mean([l.max(axis=1).sum() for l in loads]))
    sg = None if storage_price is None else storage_gamma_per_mw(storage_price)
    net = _network(net_rng, n_nodes, lf, lt, kinds, B, peak, sg)
    net.n_hvdc = int(n_hvdc)
    return Case(name=name, networks=[net], scenarios=scen, omega=omega)


def config0(seed=None) -> Case:
    """Tiny case: 6-node ring + 2 chords, 12 generators (4 gas / 4 solar /
    4 wind), 2 batteries, T = 24, one scenario."""
    return _uniform_case("tiny6", 0, 6, 12, 2, 24, 1, "ring",
                         fixed_counts=(4, 4, 4), seed=seed)


def config1(seed=None, S=16) -> Case:
    """240-node geometric network (360 lines), 1000 generators, 100
    batteries, T = 168, 16 scenarios."""
    return _uniform_case("geo240", 1, 240, 1000, 100, 168, S, "geo", seed=seed)


def config3(seed=None, S=32) -> Case:
    """500 nodes, 750 lines, 2500 generators, 250 batteries, T = 168, 32
    scenarios, carbon weight 50 $/t."""
    return _uniform_case("geo500", 3, 500, 2500, 250, 168, S, "geo", omega=50.0, seed=seed)


def config4(seed=None, S=128, storage_price=250.0) -> Case:
    """1000 nodes, 1500 lines, 5000 generators, 500 batteries, T = 168, 128
    scenarios; storage investment priced from a $/kWh capital cost."""
    return _uniform_case("geo1000", 4, 1000, 5000, 500, 168, S, "geo",
                         storage_price=storage_price, seed=seed)


def geo100(seed=None, S=16) -> Case:
    """100-node geometric network (150 lines), 417 generators, 42 batteries,
    T = 24, 16 scenarios: the size of the paper's warm-start study (Section
    3.2), with the generator and battery ratios of the other workloads."""
    return _uniform_case("geo100", 5, 100, 417, 42, 24, S, "geo", seed=seed)


def year(n_nodes=100, G=417, B=42, days=360, omega=200.0, seed=None) -> Case:
    """A synthetic year of daily scenarios (T = 24) on a geometric network of
    the warm-start study's size, for the paper's key-day study (Section 3.1,
    roughly a full year of days against a handful of key days).  The days
    differ by season as well as by weather: with y = day / days,
      load   x (1 + 0.15 cos 2 pi (y - 0.55))   (summer peak; the per-node
             lognormal level of every day is kept),
      solar  x (0.75 + 0.25 cos 2 pi (y - 0.47)) (long summer days),
      wind   x (0.8 + 0.3 cos 2 pi (y - 0.05)), clipped to 1 (windy winters),
    on top of the same hourly shapes and Beta draws as the other workloads.
    Capacity boxes are sized on the mean daily peak as elsewhere; gas emits
    0.4 t/MWh and the carbon weight defaults to 200 $/t (Section 3.1)."""
    ss = np.random.SeedSequence(9 if seed is None else seed)
    net_ss, *scen_ss = ss.spawn(days + 1)
    net_rng = np.random.Generator(np.random.PCG64(net_ss))
    lf, lt = geometric_mst_plus(net_rng, n_nodes, int(round(1.5 * n_nodes)))
    kinds = _kinds(net_rng, G)
    scen, loads = [], []
    T = 24
    for d in range(days):
        rng = np.random.Generator(np.random.PCG64(scen_ss[d]))
        y = d / days
        ld = _loads(rng, n_nodes, T) * (1.0 + 0.15 * math.cos(2 * math.pi * (y - 0.55)))
        av = _avail(rng, kinds, T)
        av[kinds == SOLAR] *= 0.75 + 0.25 * math.cos(2 * math.pi * (y - 0.47))
        av[kinds == WIND] = np.minimum(1.0, av[kinds == WIND] * (0.8 + 0.3 * math.cos(2 * math.pi * (y - 0.05))))
        ld, av = _f32(ld), _f32(av)
        loads.append(ld)
        scen.append(Scenario(network=0, T=T, avail=av, load=ld, weight=8760.0 / T))
    peak = float(np.mean([l.max(axis=1).sum() for l in loads]))
    net = _network(net_rng, n_nodes, lf, lt, kinds, B, peak)
    return Case(name=f"year{n_nodes}", networks=[net], scenarios=scen, omega=omega)


def key_days(case: Case, eta: np.ndarray, per: int = 4):
    """The paper's key days (Section 3.1 footnote): the `per` days each of
    highest peak load, highest peak net load (load minus available
    renewable capacity at the capacities eta), highest peak renewable
    availability and lowest renewable energy, taken in that order and
    skipping days already chosen.  Returns sorted scenario indices."""
    off = case.eta_offsets()
    stats = []
    for sc in case.scenarios:
        net = case.networks[sc.network]
        e = eta[off[sc.network]:off[sc.network + 1]]
        ren = net.gen_cost == 0
        load = sc.load.sum(axis=0)
        renew = (sc.avail[ren] * e[:net.n_gens][ren, None]).sum(axis=0)
        stats.append((load.max(), (load - renew).max(), renew.max(), -renew.sum()))
    stats = np.array(stats)
    chosen = []
    for col in range(4):
        for s in np.argsort(-stats[:, col], kind="stable"):
            if len([c for c in chosen if c[1] == col]) >= per:
                break
            if int(s) not in [c[0] for c in chosen]:
                chosen.append((int(s), col))
    return sorted(c[0] for c in chosen)


def config2(seed=None, S=64) -> Case:
    """64 scenarios of uneven shape: each scenario its own network with
    N ~ U{100..500}, L = 1.5N, G = round(4.17N), B = round(0.417N) and
    T drawn from {24, 72, 168}."""
    ss = np.random.SeedSequence(2 if seed is None else seed)
    nets, scens = [], []
    for s, child in enumerate(ss.spawn(S)):
        rng = np.random.Generator(np.random.PCG64(child))
        N = int(rng.integers(100, 501))
        T = int(rng.choice([24, 72, 168]))
        G = int(round(4.17 * N))
        B = int(round(0.417 * N))
        lf, lt = geometric_mst_plus(rng, N, int(round(1.5 * N)))
        kinds = _kinds(rng, G)
        ld = _loads(rng, N, T)
        av = _avail(rng, kinds, T)
        peak = float(ld.max(axis=1).sum())
        net = _network(rng, N, lf, lt, kinds, B, peak)
        nets.append(net)
        scens.append(Scenario(network=s, T=T, avail=av, load=ld, weight=8760.0 / T))
    return Case(name="uneven64", networks=nets, scenarios=scens)


def small_geo(n_nodes=12, G=30, B=3, T=24, S=2, seed=7, omega=0.0, n_hvdc=0, beta_scales=False,
              gas_ramp=0.0) -> Case:
    """A small geometric case (for quick parity tests): several tiles of
    work per class and a ragged tail at any block size.  With n_hvdc > 0
    that many HVDC links are added after the AC lines; with beta_scales the
    AC susceptances scale with line capacity; with gas_ramp > 0 every gas
    unit can move at most that share of its capacity per hour."""
    cs = _uniform_case(f"geo{n_nodes}" + (f"_hvdc{n_hvdc}" if n_hvdc else "") + ("_scaled" if beta_scales else "")
                       + (f"_ramp{gas_ramp:g}" if gas_ramp else ""),
                       100, n_nodes, G, B, T, S, "geo", omega=omega, seed=seed, n_hvdc=n_hvdc)
    net = cs.networks[0]
    net.beta_scales = bool(beta_scales)
    if gas_ramp:
        net.gen_ramp = _f32(np.where(net.gen_kind == GAS, gas_ramp, 0.0))
    return cs


def scaled_two_node(cA=20.0, cB=60.0, PA=300.0, PB=200.0, D=150.0, F=80.0, beta=10.0):
    """two_node whose line's susceptance scales with its capacity (beta at
    the capacity's lower bound F)."""
    cs = two_node(cA=cA, cB=cB, PA=PA, PB=PB, D=D, F=F, beta=beta)
    cs.networks[0].beta_scales = True
    cs.name = "scaled_two_node"
    return cs


def hvdc_two_node(cA=20.0, cB=60.0, PA=300.0, PB=200.0, D=150.0, F=80.0):
    """two_node with the line replaced by an HVDC link 0 -> 1 of capacity F:
    the flow is a free choice within [-F, F] and no angle enters."""
    cs = two_node(cA=cA, cB=cB, PA=PA, PB=PB, D=D, F=F)
    cs.networks[0].n_hvdc = 1
    cs.name = "hvdc_two_node"
    return cs


def two_node(cA=20.0, cB=60.0, PA=300.0, PB=200.0, D=150.0, F=80.0, beta=10.0, T=1):
    """Two-node network: cheap generator A at node 0 (no load), expensive
    generator B and a constant load D at node 1, one line 0 -> 1 of
    capacity F.  No batteries."""
    net = Network(
        n_nodes=2, line_from=np.array([0], np.int32), line_to=np.array([1], np.int32),
        line_beta=_f32([beta]), gen_node=np.array([0, 1], np.int32),
        gen_kind=np.array([GAS, GAS], np.int32), gen_cost=_f32([cA, cB]),
        gen_emis=_f32([GAS_EMIS, GAS_EMIS]), batt_node=np.zeros(0, np.int32),
        eta_min=_f32([PA, PB, F]), eta_max=_f32([4 * PA, 4 * PB, 4 * F]),
        gamma=_f32([1e5, 1e5, 1e5]))
    load = _f32(np.array([[0.0] * T, [D] * T]))
    sc = Scenario(network=0, T=T, avail=np.ones((2, T)), load=load, weight=8760.0 / T)
    return Case(name="two_node", networks=[net], scenarios=[sc])


def two_loads(PA=300.0, PB=200.0, F=80.0, DA=50.0, DB=150.0, cA=20.0, cB=60.0, beta=10.0):
    """Two nodes with load at both: generator A (cost cA, capacity PA) and
    load DA at node 0, generator B (cB, PB) and load DB at node 1, one line
    0 -> 1 of capacity F; T = 1, no batteries.  Capacity boxes start at the
    given values (which may be zero) and reach 400 MW above them."""
    net = Network(
        n_nodes=2, line_from=np.array([0], np.int32), line_to=np.array([1], np.int32),
        line_beta=_f32([beta]), gen_node=np.array([0, 1], np.int32),
        gen_kind=np.array([GAS, GAS], np.int32), gen_cost=_f32([cA, cB]),
        gen_emis=_f32([GAS_EMIS, GAS_EMIS]), batt_node=np.zeros(0, np.int32),
        eta_min=_f32([PA, PB, F]), eta_max=_f32([PA + 400, PB + 400, F + 400]),
        gamma=_f32([1e5, 1e5, 1e5]))
    sc = Scenario(network=0, T=1, avail=np.ones((2, 1)), load=_f32([[DA], [DB]]), weight=8760.0)
    return Case(name="two_loads", networks=[net], scenarios=[sc])


def single_node(costs, caps, D, kinds=None, T=1, avail=None):
    """One node, no lines, no batteries: the merit-order case."""
    G = len(costs)
    kinds = np.zeros(G, np.int32) if kinds is None else np.asarray(kinds, np.int32)
    net = Network(
        n_nodes=1, line_from=np.zeros(0, np.int32), line_to=np.zeros(0, np.int32),
        line_beta=np.zeros(0), gen_node=np.zeros(G, np.int32), gen_kind=kinds,
        gen_cost=_f32(costs), gen_emis=_f32(np.where(kinds == GAS, GAS_EMIS, 0.0)),
        batt_node=np.zeros(0, np.int32), eta_min=_f32(caps), eta_max=_f32(np.asarray(caps) * 4),
        gamma=_f32(np.full(G, 1e5)))
    av = np.ones((G, T)) if avail is None else _f32(avail)
    load = _f32(np.full((1, T), D) if np.isscalar(D) else np.asarray(D, float).reshape(1, T))
    sc = Scenario(network=0, T=T, avail=av, load=load, weight=8760.0 / T)
    return Case(name="single_node", networks=[net], scenarios=[sc])


def tiny_random(seed, n_nodes=2, G=2, B=1, T=2, with_line=True) -> Case:
    """Tiny random instances for brute-force enumeration."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if with_line and n_nodes >= 2:
        lf, lt = np.array([0], np.int32), np.array([1], np.int32)
    else:
        lf, lt = np.zeros(0, np.int32), np.zeros(0, np.int32)
    kinds = rng.integers(0, 3, size=G).astype(np.int32)
    kinds[0] = GAS
    load = _f32(rng.uniform(20.0, 120.0, size=(n_nodes, T)))
    av = _avail(rng, kinds, T) if T > 1 else np.ones((G, T))
    av = np.where(kinds[:, None] == GAS, 1.0, np.maximum(av, _f32(0.25)))
    av = _f32(av)
    net = Network(
        n_nodes=n_nodes, line_from=lf, line_to=lt, line_beta=_f32(rng.uniform(5, 20, size=lf.shape[0])),
        gen_node=rng.integers(0, n_nodes, size=G).astype(np.int32), gen_kind=kinds,
        gen_cost=_f32(np.where(kinds == GAS, rng.uniform(30, 80, size=G), 0.0)),
        gen_emis=_f32(np.where(kinds == GAS, GAS_EMIS, 0.0)),
        batt_node=rng.integers(0, n_nodes, size=B).astype(np.int32),
        eta_min=_f32(np.concatenate([rng.uniform(20, 80, size=G), rng.uniform(10, 50, size=lf.shape[0]),
                                     rng.uniform(5, 30, size=B)])),
        eta_max=None, gamma=None)
    net.eta_max = _f32(net.eta_min * 4)
    net.gamma = _f32(np.full(net.K, 1e5))
    sc = Scenario(network=0, T=T, avail=av, load=load, weight=8760.0 / T)
    return Case(name=f"tiny{seed}", networks=[net], scenarios=[sc])


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3, 4: config4}


def by_id(cfg: int, **kw) -> Case:
    return CONFIGS[cfg](**kw)


def jitter(eta: np.ndarray, seed: int, amount: float = 1e-2,
           eta_min: Optional[np.ndarray] = None, eta_max: Optional[np.ndarray] = None):
    """eta + U[0, amount] MW, kept inside the box (moves points off kinks)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = eta + rng.uniform(0.0, amount, size=eta.shape)
    if eta_min is not None:
        out = np.maximum(out, eta_min)
    if eta_max is not None:
        out = np.minimum(out, eta_max)
    return out
