#!/usr/bin/env python
"""Benchmark of the batched dispatch hot path on one GPU.

Default (the headline): the 1000-node workload (1000 nodes, 1500 lines,
5000 generators, 500 batteries, T = 168, 128 scenarios).  A step is one
projected-gradient planning step (Section 2.2) on a batch of scenarios
sampled from a pool: every scenario's dispatch QP solved from a cold start
to a relative KKT residual of 1e-4 (FP64 check), the implicit capacity
gradient, and the projected update.  The printed value is scenario-hours per
second over the timed steps (converged scenarios only).  Beside it: s/step
of the cold, previous-iterate and learned warm-start arms on the same
held-out planning run (network trained outside the timed region on planning
runs at other storage costs), the roofline of one ADMM iteration (the two
sweep kernels) against the HBM peak in algorithmic bytes (what one iteration
must move: every FP32 primal and dual read and written once, every
time-varying parameter read once), and
the FP64 CPU oracle timed on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "scenario-hours/s to 1e-4 KKT residual; s/gradient step, cold vs learned warm"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    0: "tiny6: 6-node ring + 2 chords, 12 generators, 2 batteries, T=24, 1 scenario",
    1: "geo240: 240 nodes, 360 lines, 1000 generators, 100 batteries, T=168, 16 scenarios",
    2: "uneven64: 64 scenarios, 100-500 nodes each, T in {24,72,168}",
    3: "geo500: 500 nodes, 750 lines, 2500 generators, 250 batteries, T=168, 32 scenarios, 50 $/t",
    4: "geo1000: 1000 nodes, 1500 lines, 5000 generators, 500 batteries, T=168, 128 scenarios",
}


def algorithmic_bytes(case, scen):
    """Bytes one launch of each sweep moves in this design (FP32 primal and
    anchor, FP64 dual anchor, FP32 dual offset):
    variable sweep: read x and the anchor x0, write x (12 B per variable),
    gather every row's FP64 anchor and FP32 offset once (12 B per row) and
    the availability profile (4 B per generator-hour);
    row sweep: read every variable once (4 B), read and write the dual offset
    (8 B per row), read the load (4 B per node-hour)."""
    nx = ny = gt = nt = 0
    for s in scen:
        sc = case.scenarios[s]
        n = case.networks[sc.network]
        T = sc.T
        nx += _n_vars(n) * T
        ny += _n_rows(n) * T
        gt += n.n_gens * T
        nt += n.n_nodes * T
    return dict(primal=12 * nx + 12 * ny + 4 * gt, dual=4 * nx + 8 * ny + 4 * nt, n_x=nx, n_y=ny)


def _n_ramped(n):
    gr = getattr(n, "gen_ramp", None)
    return 0 if gr is None else int((gr > 0).sum())


def _n_vars(n):
    """Variables per hour: outputs, flows, angles, unserved load, battery
    charge/discharge/state, ramps of ramp-limited units."""
    return n.n_gens + n.n_lines + 2 * n.n_nodes + 3 * n.n_batt + _n_ramped(n)


def _n_rows(n):
    """Equality rows per hour: balance, AC flow, SOC chain, ramp."""
    return n.n_nodes + n.n_ac + n.n_batt + _n_ramped(n)


def method_bytes(case, scen):
    """Algorithmic bytes of one ADMM iteration (what the method must move,
    not this design's layout): read and write every FP32 primal (8 n_x),
    every FP32 dual (8 n_eq), and read every time-varying FP32 parameter
    (4 (G + N) T for availability and load)."""
    tot = 0
    for s in scen:
        sc = case.scenarios[s]
        n = case.networks[sc.network]
        T = sc.T
        nx = _n_vars(n) * T
        ny = _n_rows(n) * T
        tot += 8 * nx + 8 * ny + 4 * (n.n_gens + n.n_nodes) * T
    return tot


def _read_traffic_table():
    path = os.path.join(ROOT, "profiles", "traffic.md")
    tab = {}
    if os.path.exists(path):
        with open(path) as fh:
            for line in fh:
                cells = [c.strip() for c in line.strip().strip("|").split("|")]
                if len(cells) >= 3 and cells[0].startswith("k_") and "@config" in cells[0]:
                    tab[cells[0]] = {"bytes_per_launch": float(cells[1]), "source_hash": cells[2]}
    return tab


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("gp_kernels.hip", "gp_device.h"):
        with open(os.path.join(ROOT, "paper_2410_13055_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, block, workload_id):
    """HBM bytes per launch from committed rocprofv3 counter runs (same
    kernel, block size and workload), used only while the kernel source is
    unchanged since they were taken."""
    ent = _read_traffic_table().get(f"{kernel}<{block}>@config{workload_id}")
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def _oracle_slice(sub):
    """One worker of the CPU baseline: the FP64 oracle interior point on one
    scenario slice (single-threaded BLAS), tracking the solver-independent
    KKT residual per iterate; returns (hours, seconds to the oracle's 1e-10,
    seconds to the first iterate at 1e-4 or None, iterations)."""
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    from threadpoolctl import threadpool_limits

    from oracle import dispatch as D

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        qp = D.assemble(sub, 0, sub.eta_min())
        t_asm = time.perf_counter() - t0
        sol = D.solve_ipm(qp, track=True)
        dt = time.perf_counter() - t0
    t4 = next((t for k, t in sol.history if k <= 1e-4), None)
    return sub.scenarios[0].T, dt, (None if t4 is None else t4 + t_asm), sol.iters


def cpu_baseline(case, hours=8, n_jobs=None):
    """The FP64 oracle as it stands, on the host cores: one single-threaded
    interior-point solve per process over a pool spanning every core the
    process may use, each on the first `hours` hours of a different scenario
    of the workload (capacities at their lower bounds).  The solves run side
    by side, so scenario-hours/s = (sum of hours) / the slowest worker's
    time, to the oracle's own 1e-10 and to the first iterate whose KKT
    residual reaches 1e-4."""
    import multiprocessing as mp

    from paper_2410_13055_amd import cases as C

    cores = len(os.sched_getaffinity(0))
    n = min(n_jobs or cores, len(case.scenarios))
    subs = []
    for s in range(n):
        sc = case.scenarios[s]
        h = min(hours, sc.T)
        subs.append(C.Case(name=case.name + f"-s{s}-first{h}h", networks=[case.networks[sc.network]],
                           scenarios=[C.Scenario(network=0, T=h, avail=sc.avail[:, :h].copy(),
                                                 load=sc.load[:, :h].copy(), weight=8760.0 / h)],
                           r=case.r, lambda_u=case.lambda_u, eff=case.eff, hours=case.hours, omega=case.omega))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(processes=min(cores, n)) as pool:
        res = pool.map(_oracle_slice, subs, chunksize=1)
    wall = time.perf_counter() - t0
    tot_h = sum(r[0] for r in res)
    worst10 = max(r[1] for r in res)
    t4s = [r[2] for r in res if r[2] is not None]
    worst4 = max(t4s) if len(t4s) == len(res) else None
    return {"value": round(tot_h / worst10, 3), "unit": "scenario-hours/s", "cores": min(cores, n),
            "kind": "oracle",
            "to_1e-4": {"scenario_hours_per_s": round(tot_h / worst4, 3) if worst4 else None,
                        "slowest_worker_s": round(worst4, 2) if worst4 else None},
            "to_1e-10": {"scenario_hours_per_s": round(tot_h / worst10, 3), "slowest_worker_s": round(worst10, 2)},
            "pool_wall_s": round(wall, 2),
            "sample": f"the first {hours} hours of scenarios 0..{n - 1} of the same workload at the capacities' lower "
                      f"bounds, one FP64 interior-point solve (KKT residual tracked per iterate) per process on "
                      f"{min(cores, n)} host cores; {tot_h} scenario-hours; value over the slowest worker's solve "
                      f"time to 1e-10 (the pool's wall time, process start-up included, is pool_wall_s)",
            "iterations": [r[3] for r in res]}


def summarize(stats_csv, pmc_runs, workload_id, commands):
    """Turn rocprofv3 outputs into the short text summaries kept in profiles/:
    per-kernel durations, and HBM bytes per launch of the timed sweep kernels
    from FETCH_SIZE / WRITE_SIZE (KiB per dispatch) scaled by what the same
    counters read for a 1 GiB fill (writes) and a 1 GiB sum (reads).
    pmc_runs: [(fetch_csv, write_csv, pmc_line)], one per block size.
    Returns (summary markdown, traffic table markdown)."""
    import csv
    from collections import defaultdict

    info0 = json.loads(pmc_runs[0][2])
    out = [f"# rocprofv3 summary: {info0['pmc_run']}", "", "Commands (from /tmp, TMPDIR=/tmp):", ""]
    out += [f"    {c}" for c in commands] + [""]
    out += ["## Kernel durations (--kernel-trace --stats)", "",
            "| kernel | calls | average us | total ms | share |", "|---|---|---|---|---|"]
    with open(stats_csv) as fh:
        for r in csv.DictReader(fh):
            out.append(f"| `{r['Name'][:70]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                       f"{float(r['TotalDurationNs']) / 1e6:.1f} | {float(r['Percentage']):.1f}% |")
    out += ["", "## HBM traffic per launch (--pmc FETCH_SIZE, then --pmc WRITE_SIZE)", ""]
    gib = 1 << 30
    rows = []
    for fetch_csv, write_csv, pmc_line in pmc_runs:
        info = json.loads(pmc_line)
        per = defaultdict(lambda: defaultdict(list))
        for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
            with open(path) as fh:
                for r in csv.DictReader(fh):
                    per[r["Kernel_Name"]][name].append(float(r["Counter_Value"]))

        def avg(kern_prefix, counter):
            vals = [v for k, d in per.items() if k.startswith(kern_prefix) for v in d[counter]]
            return sum(vals) / len(vals) if vals else float("nan")
        fill_w = avg("void at::native::vectorized_elementwise_kernel", "WRITE_SIZE") * 1024
        sum_r = avg("void at::native::reduce_kernel", "FETCH_SIZE") * 1024
        fw, fr = gib / fill_w, gib / sum_r
        blk = info["block"]
        out += [f"Block {blk}: calibration 1 GiB fill reads WRITE_SIZE = {fill_w / gib:.4f} GiB (write factor "
                f"{fw:.4f}); 1 GiB sum reads FETCH_SIZE = {sum_r / gib:.4f} GiB (read factor {fr:.4f}).", "",
                "| kernel | FETCH KiB | WRITE KiB | traffic bytes (scaled) | design bytes (this layout) |",
                "|---|---|---|---|---|"]
        sfx = "_q" if info.get("variant") == 2 else ""
        for kern, alg in (("k_primal" + sfx, info["primal"]), ("k_dual" + sfx, info["dual"])):
            pre = f"void gp::{kern}<{blk}, 1>"
            f_, w_ = avg(pre, "FETCH_SIZE"), avg(pre, "WRITE_SIZE")
            traffic = f_ * 1024 * fr + w_ * 1024 * fw
            out.append(f"| `{pre[len('void gp::'):]}` | {f_:.0f} | {w_:.0f} | {traffic:.0f} | {alg} |")
            rows.append((f"{kern}<{blk}>", traffic))
        out.append("")
    # the hash of the kernel sources the counter runs executed (recorded by
    # the runs themselves), so a summary written later cannot vouch for
    # kernels changed since
    hashes = {json.loads(line).get("source_hash", "unrecorded") for _, _, line in pmc_runs}
    h = hashes.pop() if len(hashes) == 1 else "mixed"
    table = ["# HBM traffic per launch of the sweep kernels", "",
             f"From the counter runs summarised in `profiles/sweeps_geo1000.md`; kernel source hash {h}.",
             "", "Table read by bench.py (valid while the kernel source hash matches):", "",
             "| key | bytes_per_launch | source_hash |", "|---|---|---|"]
    table += [f"| {k}@config{workload_id} | {t:.0f} | {h} |" for k, t in rows]
    return "\n".join(out) + "\n", "\n".join(table) + "\n"


PROFILE_COMMANDS = [
    "rocprofv3 --kernel-trace --stats --output-format csv -d <out>/prof_c4 -o run -- "
    "python3 <repo>/bench.py --steps 2 --warmup 0 --no-cpu --no-arms",
    "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/pmc_fetch_<B> -o run -- "
    "python3 <repo>/bench.py --pmc-run --pmc-block <B>      (B = 256, the roofline's launch)",
    "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/pmc_write_<B> -o run -- "
    "python3 <repo>/bench.py --pmc-run --pmc-block <B>",
    "python bench.py --summarize <out>",
]


def write_profiles(d):
    """profiles/sweeps_geo1000.md and profiles/traffic.md from the rocprofv3
    outputs of PROFILE_COMMANDS under <d>."""
    import csv
    import glob
    runs = []
    for out in sorted(glob.glob(os.path.join(d, "pmc_[0-9]*.out"))):
        if not os.path.basename(out)[4:-4].isdigit():
            continue
        blk = int(os.path.basename(out)[4:-4])
        with open(out) as fh:
            line = next(l for l in fh if l.startswith('{"pmc_run"'))
        runs.append((os.path.join(d, f"pmc_fetch_{blk}", "run_counter_collection.csv"),
                     os.path.join(d, f"pmc_write_{blk}", "run_counter_collection.csv"), line))
    summary, table = summarize(os.path.join(d, "prof_c4", "run_kernel_stats.csv"), runs, 4, PROFILE_COMMANDS)
    # the bench line of the traced run, beside the profiler's averages for the
    # same (timed) instantiations of the two sweep kernels
    with open(os.path.join(d, "prof_c4.out")) as fh:
        line = json.loads(next(l for l in fh if l.startswith('{"metric"')))
    roof = line["roofline"]
    blk = roof["launch"]["block"]
    prof = {}
    with open(os.path.join(d, "prof_c4", "run_kernel_stats.csv")) as fh:
        for r in csv.DictReader(fh):
            for k in ("k_dual", "k_primal"):
                if r["Name"].startswith(f"void gp::{k}<{blk}, 1>"):
                    prof[k] = float(r["AverageNs"]) / 1e3
    summary += ("\n## Roofline: bench.py against the profiler (same run)\n\n"
                f"bench.py (HIP events, block {blk}, 16 scenarios): k_dual {roof['ms_dual'] * 1e3:.2f} us + "
                f"k_primal {roof['ms_primal'] * 1e3:.2f} us = {roof['ms_per_iteration'] * 1e3:.2f} us per ADMM "
                f"iteration; {roof['bytes_per_iteration']} algorithmic bytes per iteration -> {roof['achieved']} GB/s, "
                f"{roof['frac'] * 100:.1f} % of 8 TB/s.  rocprofv3 averages of the same instantiations: k_dual "
                f"{prof.get('k_dual', float('nan')):.2f} us, k_primal {prof.get('k_primal', float('nan')):.2f} us.  "
                f"Headline value of that (2-step) run: {line['value']} {line['unit']}.\n")
    with open(os.path.join(ROOT, "profiles", "sweeps_geo1000.md"), "w") as fh:
        fh.write(summary)
    with open(os.path.join(ROOT, "profiles", "traffic.md"), "w") as fh:
        fh.write(table.replace("sweeps_geo240.md", "sweeps_geo1000.md"))


def write_mlp_profile(d):
    """profiles/mlp_forward_geo1000.md from <d>/prof_mlp (kernel trace of
    `bench.py --mlp`) and that run's JSON line."""
    import csv
    with open(os.path.join(d, "prof_mlp.out")) as fh:
        line = json.loads(next(l for l in fh if l.startswith('{"metric"')))
    roof = line["roofline"]
    out = ["# rocprofv3 summary: warm-start network forward, " + line["config"]["workload"], "",
           "Command (from /tmp, TMPDIR=/tmp):", "",
           "    rocprofv3 --kernel-trace --stats --output-format csv -d <out>/prof_mlp -o run -- "
           "python3 <repo>/bench.py --mlp", "",
           "| kernel | calls | average us | total ms |", "|---|---|---|---|"]
    gemm_ns, gemm_calls = 0.0, 0
    with open(os.path.join(d, "prof_mlp", "run_kernel_stats.csv")) as fh:
        for r in csv.DictReader(fh):
            out.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                       f"{float(r['TotalDurationNs']) / 1e6:.2f} |")
            if "k_gemm" in r["Name"]:
                gemm_ns += float(r["TotalDurationNs"])
                gemm_calls += int(r["Calls"])
    fwd = gemm_calls // 4
    out += ["", f"bench.py (HIP events): {roof['ms_per_forward'] * 1e3:.1f} us per forward over {roof['rows']} rows, "
            f"{roof['flops_per_forward'] / 1e9:.1f} GFLOP, {roof['achieved']} TFLOP/s = "
            f"{roof['frac'] * 100:.2f} % of the 2.5 PFLOP/s dense BF16 peak.",
            f"rocprofv3: {gemm_calls} GEMM launches = {fwd} forwards of 4 layers (one set-up call, one untimed, "
            f"the timed ones); GEMM time per forward {gemm_ns / max(fwd, 1) / 1e3:.1f} us."]
    lib = roof.get("library_reference")
    if lib:
        out += ["", "Library GEMM on the same four shapes (torch.matmul, BF16, for comparison; its kernels are the "
                "other rows of the table above): "
                f"{lib['plain_us']:.1f} us per forward as plain products ({lib['plain_tflops']} TFLOP/s = "
                f"{lib['plain_frac'] * 100:.1f} % of peak), {lib['bias_relu_us']:.1f} us with bias-add and ReLU "
                "as separate operations.", "",
                "| K | N | plain us | with bias + ReLU us |", "|---|---|---|---|"]
        out += [f"| {x['k']} | {x['n']} | {x['plain_us']} | {x['bias_relu_us']} |" for x in lib["layers"]]
    with open(os.path.join(ROOT, "profiles", "mlp_forward_geo1000.md"), "w") as fh:
        fh.write("\n".join(out) + "\n")


def write_timeline_profile(d):
    """profiles/solve_timeline_geo240.md from <d>/trace_gap (a kernel trace,
    without --stats, of one cold solve of the headline workload): how much
    of the solve the GPU is busy, and where the idle time sits."""
    import collections
    import csv
    import gzip
    path = os.path.join(d, "trace_gap", "run_kernel_trace.csv")
    fh = gzip.open(path + ".gz", "rt") if os.path.exists(path + ".gz") else open(path)
    with fh:
        ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"].split("(")[0])
                    for r in csv.DictReader(fh))
    sweeps = [e for e in ev if e[2].startswith(("void gp::k_primal<", "void gp::k_dual<")) and e[2].endswith(", 0>")]
    t0, t1 = sweeps[0][0], sweeps[-1][1]
    inside = [e for e in ev if e[0] >= t0 and e[1] <= t1]
    busy = sum(e[1] - e[0] for e in inside)
    gaps = [inside[i + 1][0] - inside[i][1] for i in range(len(inside) - 1)]
    big = [g for g in gaps if g > 20000]
    per = collections.defaultdict(lambda: [0, 0])
    for e in inside:
        per[e[2]][0] += 1
        per[e[2]][1] += e[1] - e[0]
    span = t1 - t0
    out = ["# Timeline of one cold solve: geo240, 240 nodes, 16 scenarios, T=168 (first solve of the run, "
           "autotuning included)", "",
           "Command (from /tmp, TMPDIR=/tmp):", "",
           "    rocprofv3 --kernel-trace --output-format csv -d <out>/trace_gap -o run -- "
           "python3 <repo>/bench.py --config 1 --steps 1 --warmup 0 --no-cpu --no-hbm-case",
           "    python bench.py --summarize <out>", "",
           f"From the first to the last sweep launch: {span / 1e6:.1f} ms, {len(inside)} kernels, GPU busy "
           f"{busy / 1e6:.1f} ms ({100.0 * busy / span:.1f} %).  Gaps above 20 us between kernels: {len(big)}, "
           f"{sum(big) / 1e6:.1f} ms in all (the host reading each chunk's check statistics and deciding "
           f"restarts, narrowing and graph re-captures); the rest of the idle time is spread over launch gaps "
           f"inside the replayed graphs.", "",
           "| kernel | launches | total ms | share of span |", "|---|---|---|---|"]
    for k, (c, t) in sorted(per.items(), key=lambda kv: -kv[1][1])[:10]:
        out.append(f"| `{k[:70]}` | {c} | {t / 1e6:.1f} | {100.0 * t / span:.1f} % |")
    with open(os.path.join(ROOT, "profiles", "solve_timeline_geo240.md"), "w") as fh:
        fh.write("\n".join(out) + "\n")


def write_warmstart_profile(d):
    """profiles/warmstart_geo1000.md from <d>/ws_bench.json (the JSON line of
    `bench.py --warm-start`) and its per-step log."""
    with open(os.path.join(d, "ws_bench.json")) as fh:
        r = json.loads(next(l for l in fh if l.startswith('{"metric"')))
    out = ["# s/gradient step on the 1000-node workload: cold vs learned warm vs previous-iterate warm", "",
           "Command:", "", "    python bench.py --warm-start", "",
           f"Workload: {r['config']['workload']}; tolerance {r['config']['tol']}; step size {r['config']['alpha']:.4g}.",
           "", "| arm | median s/step | s per step | max iterations per step | starts (0 cold, 1 warm, 2 screened, "
           "3 stalled) |", "|---|---|---|---|---|"]
    for arm in ("cold", "previous", "learned"):
        a = r["arms"][arm]
        out.append(f"| {arm} | {a['s_per_step_median']} | {a['s_per_step']} | {a['iterations_max_per_step']} | "
                   f"{a['starts']} |")
    t = r["training"]
    out += ["", f"Speedup (median s/step) cold / learned: {r['speedup_cold_over_learned']}; cold / previous-iterate: "
            f"{r['speedup_cold_over_previous']}.  Largest capacity difference between the learned and the cold run "
            f"after {r['steps']} steps: {r['max_eta_difference_learned_vs_cold_MW']:.3g} MW.", "",
            f"Training: planning runs under storage costs {t['storage_costs']} $/kWh, {t['steps_per_run']} steps each, "
            f"{t['rows']} rows, {t['epochs']} epochs of Adam in {t['train_s']} s (collection {t['collect_s']} s); "
            f"loss (standardised units) {t['loss_first']:.4f} -> {t['loss_last']:.4f}; network {t['network']}.", "",
            f"Network forward on {r['roofline']['rows']} rows: {r['roofline']['achieved']} TFLOP/s "
            f"({r['roofline']['frac'] * 100:.2f} % of the dense BF16 peak)."]
    with open(os.path.join(ROOT, "profiles", "warmstart_geo1000.md"), "w") as fh:
        fh.write("\n".join(out) + "\n")


def write_planwarm_profile(d):
    """profiles/plan_warm_geo100.md from the JSON lines of `bench.py
    --plan-warm` runs saved as <d>/pw_*.json (one or more carbon weights
    each, the same warm source)."""
    import glob
    rows, cfg, fails = {}, None, {"solve": 0, "step": 0}
    for f in sorted(glob.glob(os.path.join(d, "pw_*.json"))):
        with open(f) as fh:
            r = json.loads(next(l for l in fh if l.startswith('{"metric"')))
        cfg = r["config"]
        rows.update(r["by_carbon_weight"])
        for k in fails:
            fails[k] += r.get("unconverged", {}).get(k, 0)
    out = ["# Plan-level warm start (the paper's Section 3.2 study, synthetic stand-in)", "",
           "Commands:", "",
           "    python bench.py --plan-warm --pw-steps 300 --pw-src-steps 150 --pw-omegas 150 --pw-src <src.npy>",
           "    python bench.py --plan-warm --pw-steps 300 --pw-omegas 100 250 --pw-src <src.npy>", "",
           f"Workload: {cfg['workload']}; {cfg['steps']} projected-SGD steps per cold run, step "
           f"{cfg['alpha0']:.4g}/sqrt(k), the full objective evaluated every {cfg['eval_every']} steps.  The warm "
           "source is the plan after 150 steps at 200 $/t.  A run has converged at its first evaluation within "
           "2 % of the best loss of the cold run at the same carbon weight.", "",
           "| carbon weight $/t | cold steps | warm steps | speedup (cold / warm) | warm start / best cold loss | "
           "cold s | warm s |", "|---|---|---|---|---|---|---|"]
    sp = []
    for om in sorted(rows, key=float):
        r = rows[om]
        out.append(f"| {float(om):.0f} | {r['cold_steps']} | {r['warm_steps']} | "
                   f"{r['speedup']:.1f} | {r['warm_start_loss'] / r['best_cold_loss']:.4f} | {r['cold_s']} | "
                   f"{r['warm_s']} |")
        if r["speedup"]:
            sp.append(r["speedup"])
    out += ["", f"Mean speedup {sum(sp) / len(sp):.1f}x over {len(sp)} carbon weights.  Solves that missed the "
            f"tolerance in these runs: {fails['step']} step(s), {fails['solve']} evaluation(s)."]
    with open(os.path.join(ROOT, "profiles", "plan_warm_geo100.md"), "w") as fh:
        fh.write("\n".join(out) + "\n")


def hbm_case_sweeps(iters):
    """The sweep kernels on a working set far above the 256 MB Infinity
    Cache: 16 scenarios of the 1000-node workload (a GPU's share of its 128),
    timed with HIP events after a 64-iteration solve."""
    from paper_2410_13055_amd import cases, gridplan

    case = cases.config4()
    scen = list(range(16))
    plan = gridplan.Plan(case, gridplan.options(max_iter=64), stream=gridplan.current_stream())
    plan.solve(case.eta_min(), scen)
    md, mp = plan.time_sweeps(scen, iters)
    tb, tv, _, _ = plan.tuning()
    plan.close()
    ab = algorithmic_bytes(case, scen)
    sfx = "_q" if tv == 2 else ""
    res = {"workload": "geo1000, 16 of its 128 scenarios", "block": tb,
           "form": "work queue" if tv == 2 else "tile grid"}
    for k, ms, nb in (("k_primal" + sfx, mp, ab["primal"]), ("k_dual" + sfx, md, ab["dual"])):
        gbs = nb / (ms * 1e-3) / 1e9
        res[k] = {"ms_per_launch": round(ms, 5), "bytes_per_launch": nb, "achieved_GBs": round(gbs, 1),
                  "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return res


def mlp_roofline(plan, case, net, iters=20):
    """MFMA roofline of the warm-start network's forward pass on the rows of
    every scenario of the workload (one row per scenario and node), input
    features built on the device at eta_min.  Returns the roofline object."""
    import torch

    scen = list(range(len(case.scenarios)))
    rows, T = plan.nn_rows(scen)
    X = torch.empty((rows, 5 * T + 3), dtype=torch.float32, device="cuda")
    plan.features(case.eta_min(), scen, X)
    net.forward(X)
    ms = net.time_forward(rows, iters)
    flops = net.flops_per_row() * rows
    tflops = flops / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "kernel": "k_gemm (network forward: 4 GEMMs with bias/ReLU epilogues)",
            "achieved": round(tflops, 2), "peak": 2500.0, "unit": "TFLOP/s", "frac": round(tflops / 2500.0, 5),
            "traffic": None, "rows": rows, "flops_per_forward": flops, "ms_per_forward": round(ms, 5),
            "dtype": "bf16 x bf16 -> f32"}


def library_gemm_reference(rows, dims, iters=50):
    """The same layer shapes through the library GEMM (torch.matmul, BF16 in,
    hipBLASLt underneath) for comparison only: plain products, and products
    with torch's bias-add and ReLU as separate operations.  Timed with events
    on torch's current stream, which is where these products run."""
    import torch

    out = {"layers": [], "plain_us": 0.0, "bias_relu_us": 0.0}
    g = torch.Generator(device="cuda").manual_seed(0)
    flops = 0.0
    for k, n in zip(dims[:-1], dims[1:]):
        a = torch.randn(rows, k, device="cuda", dtype=torch.bfloat16, generator=g)
        w = torch.randn(k, n, device="cuda", dtype=torch.bfloat16, generator=g).contiguous()
        b = torch.randn(n, device="cuda", dtype=torch.bfloat16, generator=g)
        lay = {"k": k, "n": n}
        for key, fn in (("plain_us", lambda: a @ w), ("bias_relu_us", lambda: torch.relu(torch.addmm(b, a, w)))):
            for _ in range(3):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(iters):
                fn()
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) / iters * 1e3
            lay[key] = round(us, 1)
            out[key] += us
        flops += 2.0 * rows * k * n
        out["layers"].append(lay)
        del a, w, b
    out["plain_us"] = round(out["plain_us"], 1)
    out["bias_relu_us"] = round(out["bias_relu_us"], 1)
    out["plain_tflops"] = round(flops / (out["plain_us"] * 1e-6) / 1e12, 1)
    out["plain_frac"] = round(out["plain_tflops"] / 2500.0, 4)
    return out


def mlp_leg(args):
    """The warm-start network's forward pass alone (random weights), for its
    roofline and a profiler trace: 128 scenarios x 1000 nodes = 128,000 rows.
    Beside it, the library GEMM on the same shapes (first layer at the padded
    input width the network's kernel multiplies)."""
    from paper_2410_13055_amd import cases, gridplan

    case = cases.config4()
    plan = gridplan.Plan(case, gridplan.options(), stream=gridplan.current_stream())
    T = case.scenarios[0].T
    net = gridplan.MLP(5 * T + 3, 512, 3, 2 * T, seed=0, stream=gridplan.current_stream())
    roof = mlp_roofline(plan, case, net, args.sweep_iters)
    n_in = 5 * T + 3
    roof["library_reference"] = library_gemm_reference(roof["rows"], [(n_in + 31) // 32 * 32, 512, 512, 512, 2 * T])
    print(json.dumps({"metric": "warm-start network forward, TFLOP/s", "value": roof["achieved"],
                      "unit": "TFLOP/s", "config": {"workload": WORKLOADS[4] + "; one row per scenario and node"},
                      "roofline": roof}), flush=True)
    net.close()
    plan.close()


def plan_warm_leg(args):
    """The paper's own warm start (Section 3.2, Fig. 3 analogue): plans under
    several carbon weights, each from the no-expansion capacities (cold) and
    from the plan found at 200 $/t (warm).  Projected SGD with batches of 4
    of 16 scenarios; the full objective is evaluated on all scenarios every
    `--pw-eval` steps; a run has converged at the first evaluation within 2 %
    of the best loss of the cold run at the same weight.  Speedup = cold
    steps / warm steps."""
    import numpy as np
    import torch

    from paper_2410_13055_amd import cases, gridplan

    case = cases.geo100()
    S = len(case.scenarios)
    pool = list(range(S))
    lo, hi = case.eta_min(), case.eta_max()
    gamma = case.gamma()
    w = np.array([sc.weight for sc in case.scenarios])
    log = lambda *a: print("[plan-warm]", *a, file=sys.stderr, flush=True)  # noqa: E731
    # batches change every step: a fixed sweep configuration skips re-tuning
    plan = gridplan.Plan(case, gridplan.options(block=256, variant=1, check_every=64),
                         stream=gridplan.current_stream())

    fails = {"solve": 0, "step": 0}

    def phi(eta, omega):
        _, st, rc = plan.solve(eta, pool, warm=1)
        if rc:
            fails["solve"] += 1
            log(f"evaluation solve not converged: {[(x['iters'], x['kkt'], x['start']) for x in st if x['status']]}")
        h = np.array([x["cost"] + omega * x["emis"] for x in st])
        return float(gamma @ eta + np.mean(w * h))

    plan.solve(lo, pool[:4], warm=0)
    g0, _, _ = plan.grad(pool[:4], 200.0)
    alpha = 0.1 * float((hi - lo).min()) / float(np.abs(gamma + g0).max())

    def run(eta0, omega, steps, seed, target=None):
        # step alpha / sqrt(k): the sampled gradients are noisy and span
        # three orders of magnitude across capacities
        rng = np.random.default_rng(seed)
        eta = eta0.copy()
        curve = [(0, phi(eta, omega))]
        t0 = time.perf_counter()
        for k in range(1, steps + 1):
            scen = sorted(rng.choice(pool, 4, replace=False).tolist())
            eta, _, _, rc = plan.step(alpha / np.sqrt(k), scen, gamma, eta, omega=omega, warm=1)
            if rc:
                fails["step"] += 1
                log(f"step {k}: solve or adjoint not converged (rc {rc})")
            if k % args.pw_eval == 0:
                curve.append((k, phi(eta, omega)))
                log(f"omega {omega} step {k}: objective {curve[-1][1]:.6e}")
                if target is not None and curve[-1][1] <= target:
                    break
        torch.cuda.synchronize()
        return eta, curve, time.perf_counter() - t0

    def first_within(curve, best):
        return next(k for k, v in curve if v <= 1.02 * best)

    if args.pw_src and os.path.exists(args.pw_src):
        src = np.load(args.pw_src)
        log(f"step size {alpha:.4g}; warm source read from {args.pw_src}")
    else:
        log(f"step size {alpha:.4g}; cold run at 200 $/t, the warm source")
        src, curve200, _ = run(lo, 200.0, args.pw_src_steps or args.pw_steps, 200)
        if args.pw_src:
            np.save(args.pw_src, src)
    res = {}
    for omega in args.pw_omegas:
        _, cc, tc = run(lo, omega, args.pw_steps, int(omega))
        best = min(v for _, v in cc)
        kc = first_within(cc, best)
        _, wc, tw = run(src, omega, args.pw_steps, int(omega) + 1, target=1.02 * best)
        kw = next((k for k, v in wc if v <= 1.02 * best), None)
        res[str(omega)] = {"cold_steps": kc, "warm_steps": kw, "best_cold_loss": best,
                           "warm_start_loss": wc[0][1], "speedup": (kc / kw) if kw else None,
                           "cold_s": round(tc, 2), "warm_s": round(tw, 2)}
        log(f"omega {omega}: cold {kc} steps, warm {kw} steps (warm start at {wc[0][1] / best:.4f} of the best)")
    sp = [r["speedup"] for r in res.values() if r["speedup"]]
    out = {"metric": "planning steps to within 2 % of the best cold loss, cold / warm (plan-level warm start)",
           "value": round(float(np.mean(sp)), 2) if sp else None, "unit": "x",
           "config": {"workload": "geo100: 100 nodes, 150 lines, 417 generators, 42 batteries, T=24, "
                                  "16 scenarios; SGD batches of 4; warm from the 200 $/t plan",
                      "steps": args.pw_steps, "eval_every": args.pw_eval, "alpha0": alpha,
                      "step_rule": "alpha0 / sqrt(k)"},
           "by_carbon_weight": res, "unconverged": fails}
    plan.close()
    print(json.dumps(out), flush=True)


def key_days_leg(args):
    """The paper's key-day study (Section 3.1, Fig. 2 analogue) on a synthetic
    360-day year of the 100-node stand-in at 200 $/t: projected SGD with
    batches of B = 8 days sampled from 16 key days (top 4 peak load, peak net
    load, peak renewable and lowest renewable days) or from all 360 days,
    the same number of steps for both, every run's plan scored on all 360
    days (out of sample for the key-day run) every `--kd-eval` steps."""
    import numpy as np
    import torch

    from paper_2410_13055_amd import cases, gridplan

    case = cases.year()
    S = len(case.scenarios)
    full = list(range(S))
    lo, hi = case.eta_min(), case.eta_max()
    gamma = case.gamma()
    omega = case.omega
    keyd = cases.key_days(case, lo)
    log = lambda *a: print("[key-days]", *a, file=sys.stderr, flush=True)  # noqa: E731
    plan = gridplan.Plan(case, gridplan.options(block=256, variant=1, check_every=64),
                         stream=gridplan.current_stream())
    fails = {"eval": 0, "step": 0}

    def phi_full(eta):
        _, st, rc = plan.solve(eta, full, warm=1)
        if rc:
            fails["eval"] += 1
        return float(gamma @ eta + plan.objective(full, omega, eta=eta))

    plan.solve(lo, keyd[:args.kd_batch], warm=0)
    g0, _, _ = plan.grad(keyd[:args.kd_batch], omega)
    alpha = 0.1 * float((hi - lo).min()) / float(np.abs(gamma + g0).max())
    log(f"key days {keyd}; step size {alpha:.4g}/sqrt(k)")

    def run(pool, seed, label):
        rng = np.random.default_rng(seed)
        eta = lo.copy()
        curve = [(0, phi_full(eta))]
        t0 = time.perf_counter()
        for k in range(1, args.kd_steps + 1):
            scen = sorted(rng.choice(pool, args.kd_batch, replace=False).tolist())
            eta, _, _, rc = plan.step(alpha / np.sqrt(k), scen, gamma, eta, omega=omega, warm=1)
            if rc:
                fails["step"] += 1
            if k % args.kd_eval == 0:
                curve.append((k, phi_full(eta)))
                log(f"{label} step {k}: 360-day objective {curve[-1][1]:.6e}")
        torch.cuda.synchronize()
        return eta, curve, round(time.perf_counter() - t0, 1)

    out = {"metric": "360-day objective of the plan: key-day SGD vs full-year SGD (lower is better)",
           "config": {"workload": f"year100: {case.networks[0].n_nodes} nodes, {case.networks[0].n_lines} lines, "
                                  f"{case.networks[0].n_gens} generators, {case.networks[0].n_batt} batteries, "
                                  f"T=24, {S} daily scenarios, 200 $/t",
                      "batch": args.kd_batch, "steps": args.kd_steps, "eval_every": args.kd_eval,
                      "alpha0": alpha, "step_rule": "alpha0 / sqrt(k)", "key_days": keyd}}
    # the two runs are independent (each starts from eta_min with its own
    # sampling seed), so they may be made in separate processes
    if args.kd_arm in ("key", "both"):
        _, out["key_days_curve"], out["key_days_s"] = run(keyd, 1, "key days")
    if args.kd_arm in ("full", "both"):
        _, out["full_year_curve"], out["full_year_s"] = run(full, 2, "full year")
    out["unconverged"] = fails
    plan.close()
    print(json.dumps(out), flush=True)


def write_keydays_profile(d):
    """profiles/key_days_year100.md from the lines of `bench.py --key-days`
    in <d>: kd.json (both runs), or kd_key.json and kd_full.json (one run
    each, `--kd-arm key` / `--kd-arm full`)."""
    r = {}
    for name in ("kd.json", "kd_key.json", "kd_full.json"):
        if os.path.exists(os.path.join(d, name)):
            with open(os.path.join(d, name)) as fh:
                part = json.loads(next(l for l in fh if l.startswith('{"metric"')))
            fails = {k: v + r.get("unconverged", {}).get(k, 0) for k, v in part.pop("unconverged").items()}
            r.update(part)
            r["unconverged"] = fails
    if "key_days_curve" not in r or "full_year_curve" not in r:
        return
    fk, ff = r["key_days_curve"][-1][1], r["full_year_curve"][-1][1]
    r["value"] = (fk - ff) / fk
    c = r["config"]
    out = ["# Key days vs the full year (the paper's Section 3.1 study, synthetic stand-in)", "",
           "Commands:", "", f"    python bench.py --key-days --kd-steps {c['steps']} --kd-arm key",
           f"    python bench.py --key-days --kd-steps {c['steps']} --kd-arm full", "",
           f"Workload: {c['workload']}; projected SGD, batches of {c['batch']} days, {c['steps']} steps per run, "
           f"step {c['alpha0']:.4g}/sqrt(k); both plans scored on all days every {c['eval_every']} steps.  Key days "
           f"(top 4 peak load, peak net load, peak renewable, lowest renewable): {c['key_days']}.", "",
           "| step | 360-day objective, key-day run | 360-day objective, full-year run |", "|---|---|---|"]
    for (k, a), (_, b) in zip(r["key_days_curve"], r["full_year_curve"]):
        out.append(f"| {k} | {a:.6e} | {b:.6e} |")
    rel = 100 * r["value"]
    out += ["", f"At the last evaluation the full-year plan's 360-day objective is {abs(rel):.2f} % "
            f"{'below' if rel >= 0 else 'above'} the key-day plan's (run times, evaluations included: "
            f"{r['key_days_s']:.1f} s and {r['full_year_s']:.1f} s).  Solves that missed the tolerance: "
            f"{r['unconverged']}."]
    with open(os.path.join(ROOT, "profiles", "key_days_year100.md"), "w") as fh:
        fh.write("\n".join(out) + "\n")


def warm_start_leg(args):
    """s/gradient step on the 1000-node workload, cold vs learned warm (with
    the previous-iterate warm start as the extra baseline).

    Protocol (projected SGD as in Section 3.2: a pool of scenarios, a batch
    sampled per step): training data come from planning runs under four
    storage capital costs; the held-out run uses a fifth cost.  Every arm
    of the held-out run samples the same batches; a step is solve (to the
    1e-4 KKT residual) + gradient + projected update, timed end to end, the
    learned arm including feature extraction, inference and seeding."""
    import numpy as np
    import torch

    from paper_2410_13055_amd import cases, gridplan
    from paper_2410_13055_amd.warmstart import LearnedWarmStart

    case = cases.config4()
    net = case.networks[0]
    G, L, N, T = net.n_gens, net.n_lines, net.n_nodes, case.scenarios[0].T
    pool, B, steps = list(range(args.ws_pool)), args.ws_batch, args.ws_steps
    lo, hi = case.eta_min(), case.eta_max()
    log = lambda *a: print("[warm]", *a, file=sys.stderr, flush=True)  # noqa: E731

    def gamma_for(price):
        g = case.gamma().copy()
        g[G + L:] = cases.storage_gamma_per_mw(price)
        return g

    def batches(seed):
        rng = np.random.default_rng(seed)
        return [sorted(rng.choice(pool, B, replace=False).tolist()) for _ in range(steps)]

    # one tuning pass fixes the sweep configuration for every plan
    probe = gridplan.Plan(case, gridplan.options(max_iter=64), stream=gridplan.current_stream())
    probe.solve(lo, pool[:B])
    tb, tv, tce, _ = probe.tuning()
    probe.close()
    opts = dict(block=tb, variant=tv, check_every=tce)
    log(f"sweep configuration: block {tb}, form {tv}, {tce} iterations per replay")

    plan = gridplan.Plan(case, gridplan.options(**opts), stream=gridplan.current_stream())
    ws = LearnedWarmStart(plan, T, seed=0)
    held_price = args.ws_held_price
    plan.solve(lo, pool[:B], warm=0)
    g0, _, _ = plan.grad(pool[:B])
    alpha = 0.05 * float((hi - lo).min()) / float(np.abs(gamma_for(held_price) + g0).max())

    def run(p, price, seed, arm, collect=False):
        gam = gamma_for(price)
        eta = lo.copy()
        out = {"s": [], "iters": [], "starts": [], "kkt": []}
        for k, scen in enumerate(batches(seed)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if arm == "learned":
                ws.seed(eta, scen)
            _, st, rc = p.solve(eta, scen, warm=0 if arm == "cold" else 1)
            g, _, _ = p.grad(scen)
            if collect:
                ws.collect(eta, scen)
            eta = np.clip(eta - alpha * (gam + g), lo, hi)
            torch.cuda.synchronize()
            out["s"].append(time.perf_counter() - t0)
            out["iters"].append(max(x["iters"] for x in st))
            out["starts"] += [x["start"] for x in st]
            out["kkt"].append(max(x["kkt"] for x in st))
            log(f"{arm} price {price} step {k}: {out['s'][-1]:.2f} s, iterations {out['iters'][-1]}, "
                f"starts {[x['start'] for x in st]}")
        out["eta"] = eta
        return out

    t0 = time.perf_counter()
    for i, price in enumerate(args.ws_train_prices):
        run(plan, price, 100 + i, "previous", collect=True)
    collect_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    losses = ws.train(epochs=args.ws_epochs, batch_rows=4096, lr=1e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log(f"trained on {ws.rows} rows: loss {losses[0]:.4f} -> {losses[-1]:.4f} in {train_s:.1f} s")

    arms = {}
    for arm in ("cold", "previous", "learned"):
        p = plan if arm == "learned" else gridplan.Plan(case, gridplan.options(**opts),
                                                        stream=gridplan.current_stream())
        arms[arm] = run(p, held_price, 999, arm)
        if p is not plan:
            p.close()
    # inference GEMMs: MFMA roofline of the trained network's forward pass
    # on the rows of all 128 scenarios
    roof = mlp_roofline(plan, case, ws.net)
    plan.close()

    def summary(a):
        return {"s_per_step_median": round(float(np.median(a["s"])), 4),
                "s_per_step": [round(x, 3) for x in a["s"]],
                "iterations_max_per_step": a["iters"],
                "starts": {str(k): a["starts"].count(k) for k in sorted(set(a["starts"]))},
                "kkt_max": float(max(a["kkt"]))}
    med = {k: float(np.median(v["s"])) for k, v in arms.items()}
    drift = float(np.abs(arms["learned"]["eta"] - arms["cold"]["eta"]).max())
    out = {
        "metric": "s/gradient step, cold vs learned warm",
        "value": round(med["learned"], 4),
        "unit": "s/step",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": round(med["learned"] * 1e3, 1),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 solve / bf16 MLP",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[4] + f"; batch of {B} sampled per step from the first "
                               f"{len(pool)} scenarios; held-out storage cost {held_price} $/kWh",
                   "tol": 1e-4, "alpha": alpha},
        "speedup_cold_over_learned": round(med["cold"] / med["learned"], 3),
        "speedup_cold_over_previous": round(med["cold"] / med["previous"], 3),
        "arms": {k: summary(v) for k, v in arms.items()},
        "max_eta_difference_learned_vs_cold_MW": drift,
        "training": {"storage_costs": args.ws_train_prices, "steps_per_run": steps, "rows": ws.rows,
                     "epochs": args.ws_epochs, "loss_first": losses[0], "loss_last": losses[-1],
                     "collect_s": round(collect_s, 1), "train_s": round(train_s, 2),
                     "network": f"{5 * T + 3} -> 512 x3 -> {2 * T}, {ws.net.n_params} parameters"},
        "roofline": roof,
    }
    print(json.dumps(out), flush=True)


def headline_leg(args):
    """The headline line on the 1000-node workload (see the module
    docstring).  Projected SGD as in Section 3.2: a pool of scenarios, a
    batch of B sampled per step, step alpha; the held-out planning run uses
    a storage capital cost of 250 $/kWh.

    Timed: K cold planning steps.  Untimed beside them (while the run's time
    budget allows): the previous-iterate and learned warm-start arms on the
    first M steps of the same batch sequence, the network trained on
    planning runs at other storage costs, the sweep roofline, the network's
    MFMA roofline and the CPU oracle."""
    import numpy as np
    import torch

    from paper_2410_13055_amd import cases, gridplan
    from paper_2410_13055_amd.warmstart import LearnedWarmStart

    t_start = time.perf_counter()
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)  # noqa: E731
    case = cases.config4()
    net = case.networks[0]
    G, L, N, T = net.n_gens, net.n_lines, net.n_nodes, case.scenarios[0].T
    pool, B = list(range(args.pool)), args.batch
    lo, hi = case.eta_min(), case.eta_max()
    log(f"{WORKLOADS[4]}: case built in {time.perf_counter() - t_start:.1f} s")

    def gamma_for(price):
        g = case.gamma().copy()
        g[G + L:] = cases.storage_gamma_per_mw(price)
        return g

    def batches(seed, n):
        rng = np.random.default_rng(seed)
        return [sorted(rng.choice(pool, B, replace=False).tolist()) for _ in range(n)]

    probe = gridplan.Plan(case, gridplan.options(max_iter=64), stream=gridplan.current_stream())
    probe.solve(lo, pool[:B])
    tb, tv, tce, _ = probe.tuning()
    probe.close()
    opts = dict(block=tb, variant=tv, check_every=tce)
    log(f"sweep configuration: block {tb}, form {tv}, {tce} iterations per replay")
    plan = gridplan.Plan(case, gridplan.options(**opts), stream=gridplan.current_stream())
    held = args.ws_held_price
    gam = gamma_for(held)
    state = {"alpha": None}

    def step(p, eta, scen, arm, ws=None, collect=None):
        if arm == "learned":
            ws.seed(eta, scen)
        _, st, rc = p.solve(eta, scen, warm=0 if arm == "cold" else 1)
        g, _, rc2 = p.grad(scen, eta=eta)
        if collect is not None:
            collect.collect(eta, scen)
        if state["alpha"] is None:  # step size from the first gradient (a share of the smallest box)
            state["alpha"] = 0.05 * float((hi - lo).min()) / float(np.abs(gam + g).max())
        return np.clip(eta - state["alpha"] * (gam + g), lo, hi), st, rc, rc2

    def run_arm(p, arm, bl, price=None, ws=None, collect=None, label=""):
        eta = lo.copy()
        out = {"s": [], "iters": [], "starts": [], "unconverged": 0, "kkt": []}
        for k, scen in enumerate(bl):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eta, st, rc, rc2 = step(p, eta, scen, arm, ws, collect)
            torch.cuda.synchronize()
            out["s"].append(time.perf_counter() - t0)
            out["iters"].append(max(x["iters"] for x in st))
            out["starts"] += [x["start"] for x in st]
            out["unconverged"] += sum(1 for x in st if x["status"])
            out["kkt"].append(max(x["kkt"] for x in st))
            log(f"{label or arm} step {k}: {out['s'][-1]:.2f} s, iterations {out['iters'][-1]}, "
                f"starts {[x['start'] for x in st]}")
        out["eta"] = eta
        return out

    # warm-up: W cold steps of another batch sequence
    run_arm(plan, "cold", batches(7, args.warmup), label="warmup")
    torch.cuda.synchronize()
    # timed: K cold steps of the held-out run
    held_batches = batches(999, args.steps)
    t0 = time.perf_counter()
    cold = run_arm(plan, "cold", held_batches, label="cold (timed)")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    conv_h = args.steps * B * T - cold["unconverged"] * T
    value = conv_h / elapsed
    log(f"timed {args.steps} steps in {elapsed:.1f} s: {value:.1f} scenario-hours/s")

    def left():
        return args.budget - (time.perf_counter() - t_start)

    per_step = elapsed / args.steps
    M = min(args.arm_steps, args.steps)
    arms = {"cold": cold}
    training = None
    roof_mlp = None
    # training data (previous-iterate planning runs at other storage costs),
    # then the two warm arms; each piece runs only while the budget allows it
    Mc = args.collect_steps
    need_collect = len(args.ws_train_prices) * Mc * per_step * 1.1
    if args.arms and left() > need_collect + 2 * M * per_step + 60:
        ws = LearnedWarmStart(plan, T, seed=0)
        t1 = time.perf_counter()
        for i, price in enumerate(args.ws_train_prices):
            gam_keep = gam
            gam = gamma_for(price)
            run_arm(plan, "previous", batches(100 + i, Mc), collect=ws, label=f"collect {price}")
            gam = gam_keep
        collect_s = time.perf_counter() - t1
        t1 = time.perf_counter()
        losses = ws.train(epochs=args.ws_epochs, batch_rows=4096, lr=1e-3)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t1
        training = {"storage_costs": args.ws_train_prices, "steps_per_run": Mc, "batch": B, "rows": ws.rows,
                    "epochs": args.ws_epochs, "loss_first": losses[0], "loss_last": losses[-1],
                    "collect_s": round(collect_s, 1), "train_s": round(train_s, 2),
                    "network": f"{5 * T + 3} -> 512 x3 -> {2 * T}, {ws.net.n_params} parameters"}
        log(f"trained on {ws.rows} rows in {train_s:.1f} s: loss {losses[0]:.4f} -> {losses[-1]:.4f}")
        if left() > 2 * M * per_step + 30:
            prev_plan = gridplan.Plan(case, gridplan.options(**opts), stream=gridplan.current_stream())
            arms["previous"] = run_arm(prev_plan, "previous", held_batches[:M])
            prev_plan.close()
            arms["learned"] = run_arm(plan, "learned", held_batches[:M], ws=ws)
        roof_mlp = mlp_roofline(plan, case, ws.net)
    plan.close()

    # one ADMM iteration against the HBM peak: 16 scenarios (a GPU's share of
    # 128 on 8 GPUs; 3 GB resident, far above the 256 MB Infinity Cache)
    # (the tile grid at 256 threads, the launch the counter runs measure)
    scen16 = list(range(16))
    p16 = gridplan.Plan(case, gridplan.options(max_iter=64, block=256, variant=1, check_every=64),
                        stream=gridplan.current_stream())
    p16.solve(lo, scen16)
    md, mp_ = p16.time_sweeps(scen16, args.sweep_iters)
    tb16, tv16, _, _ = p16.tuning()
    p16.close()
    ab = algorithmic_bytes(case, scen16)
    bm = method_bytes(case, scen16)
    it_ms = md + mp_
    achieved = bm / (it_ms * 1e-3) / 1e9
    sfx = "_q" if tv16 == 2 else ""
    tp = measured_traffic("k_primal" + sfx, tb16, 4)
    td = measured_traffic("k_dual" + sfx, tb16, 4)
    roof = {"bound": "hbm", "kernel": f"k_dual{sfx} + k_primal{sfx} (one ADMM iteration)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (tp + td) if (tp is not None and td is not None) else None,
            "bytes_per_iteration": bm, "design_bytes_per_iteration": ab["primal"] + ab["dual"],
            "ms_per_iteration": round(it_ms, 5), "ms_dual": round(md, 5), "ms_primal": round(mp_, 5),
            "launch": {"scenarios": 16, "block": tb16, "form": "work queue" if tv16 == 2 else "tile grid"}}

    def med(a, n=None):
        v = a["s"][:n] if n else a["s"]
        return round(float(np.median(v)), 4)

    arm_out = {k: {"s_per_step_median": med(v, M), "s_per_step": [round(x, 3) for x in v["s"][:M]],
                   "iterations_max_per_step": v["iters"][:M],
                   "starts": {str(q): v["starts"][:M * B].count(q) for q in sorted(set(v["starts"][:M * B]))},
                   "unconverged": v["unconverged"]} for k, v in arms.items()}
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "scenario-hours/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[4] + f"; cold planning steps on batches of {B} sampled from the first "
                               f"{len(pool)} scenarios; storage cost {held} $/kWh",
                   "batch": B, "pool": len(pool), "scenario_hours_per_step": B * T, "start": "cold", "tol": 1e-4},
        "roofline": roof,
        "s_per_gradient_step": {"first_steps": M, "arms": arm_out,
                                "speedup_cold_over_learned": (round(med(cold, M) / arm_out["learned"]["s_per_step_median"], 3)
                                                              if "learned" in arm_out else None),
                                "speedup_cold_over_previous": (round(med(cold, M) / arm_out["previous"]["s_per_step_median"], 3)
                                                               if "previous" in arm_out else None),
                                "training": training},
        "extra": {"cold_s_per_step_median": med(cold), "iters_max": int(max(cold["iters"])),
                  "kkt_max": float(max(cold["kkt"])), "unconverged_scenarios": cold["unconverged"],
                  "mlp_roofline": roof_mlp},
    }
    if args.cpu and left() > 60:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_hours)
    log(f"total {time.perf_counter() - t_start:.1f} s")
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4, choices=sorted(WORKLOADS),
                    help="4 (default): the headline line; others: cold solves of every scenario per step")
    ap.add_argument("--no-cpu", dest="cpu", action="store_false", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-hours", type=int, default=8)
    ap.add_argument("--batch", type=int, default=4, help="scenarios per planning step (headline)")
    ap.add_argument("--pool", type=int, default=16, help="scenarios the batches are drawn from (headline)")
    ap.add_argument("--arm-steps", type=int, default=10, help="steps of the warm-start arms (headline)")
    ap.add_argument("--collect-steps", type=int, default=6,
                    help="steps of each planning run that collects the network's training data (headline)")
    ap.add_argument("--no-arms", dest="arms", action="store_false",
                    help="headline: skip the warm-start arms and their training (profiled runs)")
    ap.add_argument("--budget", type=float, default=600.0,
                    help="seconds after which the headline run skips its untimed extras")
    ap.add_argument("--sweep-iters", type=int, default=50)
    ap.add_argument("--pmc-block", type=int, default=256, choices=[128, 256, 512],
                    help="block size of the sweeps in --pmc-run")
    ap.add_argument("--pmc-run", action="store_true",
                    help="short run for hardware counters: one iteration chunk, 10 timed sweeps of "
                         "each kernel and a 1 GiB device copy that calibrates the byte counters")
    ap.add_argument("--no-hbm-case", dest="hbm_case", action="store_false",
                    help="skip timing the sweeps on 16 scenarios of the 1000-node workload")
    ap.add_argument("--plan-warm", action="store_true",
                    help="the paper's plan-level warm start on a 100-node case (cold vs warm planning steps)")
    ap.add_argument("--pw-steps", type=int, default=200)
    ap.add_argument("--pw-eval", type=int, default=5)
    ap.add_argument("--pw-omegas", type=float, nargs="+", default=[100.0, 150.0, 250.0, 300.0])
    ap.add_argument("--pw-src", help="file of the 200 $/t plan: read when present, else written")
    ap.add_argument("--pw-src-steps", type=int, default=0, help="steps of the 200 $/t run (default --pw-steps)")
    ap.add_argument("--key-days", action="store_true",
                    help="the key-day study: 16 key days vs the full year of the 100-node stand-in")
    ap.add_argument("--kd-steps", type=int, default=100)
    ap.add_argument("--kd-eval", type=int, default=25)
    ap.add_argument("--kd-batch", type=int, default=8)
    ap.add_argument("--kd-arm", choices=("key", "full", "both"), default="both",
                    help="which SGD run of the key-day study to make")
    ap.add_argument("--mlp", action="store_true",
                    help="time the warm-start network's forward pass on 128,000 rows (its MFMA roofline)")
    ap.add_argument("--warm-start", action="store_true",
                    help="s/gradient step on the 1000-node workload: cold vs learned warm vs previous-iterate")
    ap.add_argument("--ws-pool", type=int, default=16)
    ap.add_argument("--ws-batch", type=int, default=4)
    ap.add_argument("--ws-steps", type=int, default=10)
    ap.add_argument("--ws-epochs", type=int, default=150)
    ap.add_argument("--ws-train-prices", type=float, nargs="+", default=[100.0, 400.0])
    ap.add_argument("--ws-held-price", type=float, default=250.0)
    ap.add_argument("--summarize", metavar="DIR",
                    help="write profiles/sweeps_geo240.md and profiles/traffic.md from the rocprofv3 outputs "
                         "under DIR (prof_c1/, pmc_fetch_<block>/, pmc_write_<block>/, pmc_<block>.out)")
    args = ap.parse_args()
    if args.summarize:
        if os.path.exists(os.path.join(args.summarize, "prof_c4")):
            write_profiles(args.summarize)
        if os.path.exists(os.path.join(args.summarize, "prof_mlp")):
            write_mlp_profile(args.summarize)
        if os.path.exists(os.path.join(args.summarize, "ws_bench.json")):
            write_warmstart_profile(args.summarize)
        if any(os.path.exists(os.path.join(args.summarize, n)) for n in ("kd.json", "kd_key.json")):
            write_keydays_profile(args.summarize)
        if os.path.exists(os.path.join(args.summarize, "trace_gap")):
            write_timeline_profile(args.summarize)
        import glob
        if glob.glob(os.path.join(args.summarize, "pw_*.json")):
            write_planwarm_profile(args.summarize)
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; multi-GPU runs are not part of it "
              "(scenarios would shard across GPUs with one all-reduce of the gradient per step)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2410_13055_amd import cases, gridplan

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.warm_start:
        warm_start_leg(args)
        return
    if args.mlp:
        mlp_leg(args)
        return
    if args.plan_warm:
        plan_warm_leg(args)
        return
    if args.key_days:
        key_days_leg(args)
        return
    if args.config == 4 and not args.pmc_run:
        headline_leg(args)
        return
    case = cases.by_id(args.config)
    # the counter run on the headline workload measures the roofline's batch:
    # 16 of its scenarios
    scen = list(range(16 if args.config == 4 else len(case.scenarios)))
    sh = case.scenario_hours(scen)
    eta = case.eta_min()
    omega = case.omega
    print(f"[bench] {WORKLOADS[args.config]}", file=sys.stderr, flush=True)
    if args.pmc_run:
        plan = gridplan.Plan(case, gridplan.options(max_iter=64, block=args.pmc_block, variant=1, check_every=64),
                             stream=gridplan.current_stream())
        plan.solve(eta, scen, warm=0)
        md, mp = plan.time_sweeps(scen, 10)
        tb, tv, tce, _ = plan.tuning()
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)  # 1 GiB read + 1 GiB written
        total = a.sum()  # reduction kernel: 1 GiB read (calibrates the read counter)
        torch.cuda.synchronize()
        assert float(total) == float(1 << 28)
        ab = algorithmic_bytes(case, scen)
        print(json.dumps({"pmc_run": WORKLOADS[args.config] + f" (sweeps over {len(scen)} scenarios)",
                          "ms_dual": md, "ms_primal": mp, "block": tb, "variant": tv, "copy_bytes": 1 << 30,
                          "method_bytes_per_iteration": method_bytes(case, scen),
                          "source_hash": kernel_source_hash(), **ab}), flush=True)
        plan.close()
        return
    plan = gridplan.Plan(case, gridplan.options(), stream=gridplan.current_stream())
    for w in range(args.warmup):
        _, st, _ = plan.solve(eta, scen, warm=0)
        plan.grad(scen, omega)
        print(f"[bench] warmup {w} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    iters, kkts, solve_s, grad_s = [], [], 0.0, 0.0
    t0 = time.perf_counter()
    for k in range(args.steps):
        a = time.perf_counter()
        cost, st, rc = plan.solve(eta, scen, warm=0)
        b = time.perf_counter()
        g, hval, rc2 = plan.grad(scen, omega)
        c = time.perf_counter()
        solve_s += b - a
        grad_s += c - b
        iters += [s["iters"] for s in st]
        kkts += [s["kkt"] for s in st]
        print(f"[bench] step {k}: solve {b - a:.3f} s grad {c - b:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ms_step = elapsed / args.steps * 1e3

    # dominant kernel: HIP-event durations of the two sweeps on the plan's stream
    md, mp = plan.time_sweeps(scen, args.sweep_iters)
    tb, tv, tce, _ = plan.tuning()
    sfx = "_q" if tv == 2 else ""
    # one ADMM iteration (row sweep + variable sweep) in algorithmic bytes
    # (method_bytes); a working set that fits the 256 MB Infinity Cache
    # makes the rate an effective one, not an HBM one
    ab = algorithmic_bytes(case, scen)
    bm = method_bytes(case, scen)
    ms = md + mp
    achieved = bm / (ms * 1e-3) / 1e9
    resident = ab["primal"] + ab["dual"]
    roof = {"bound": "hbm" if resident > 256e6 else "effective", "kernel": "k_dual + k_primal (one ADMM iteration)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None, "bytes_per_iteration": bm, "design_bytes_per_iteration": resident,
            "ms_per_iteration": round(ms, 5), "ms_dual": round(md, 5), "ms_primal": round(mp, 5),
            "launch": {"block": tb, "form": "work queue" if tv == 2 else "tile grid",
                       "iterations_per_replay": tce}}
    plan.close()

    out = {
        "metric": METRIC,
        "value": round(args.steps * sh / elapsed, 2),
        "unit": "scenario-hours/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "scenarios": len(scen), "scenario_hours": sh,
                   "start": "cold", "tol": 1e-4, "omega": omega},
        "roofline": roof,
        "extra": {"solve_s_per_step": round(solve_s / args.steps, 4),
                  "grad_s_per_step": round(grad_s / args.steps, 4),
                  "iters_mean": float(np.mean(iters)), "iters_max": int(np.max(iters)),
                  "kkt_max": float(np.max(kkts)),
                  "solve_only_scenario_hours_per_s": round(args.steps * sh / solve_s, 2)},
    }
    if args.hbm_case:
        out["extra"]["hbm_case"] = hbm_case_sweeps(args.sweep_iters)
    if args.cpu:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_hours)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
