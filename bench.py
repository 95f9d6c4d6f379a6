"""Benchmark of the PAKR hot path on one MI355X.

A step is one AO-x query of the 3D double-integrator workload (6D state, 30
random boxes in [0,10]^3, B 4096, A 8, T 20, dt 0.05, tree capacity 262144,
duration cost) run on the device for a 200 ms budget: every iteration of
every round samples, searches the tree, rolls out, checks, prunes and inserts
on the GPU.  Each step uses its own scene and Philox seed; all plans are
created (inputs resident in HBM) before the timed region.

Printed: one JSON line with expansions/s over the timed steps, time to first
and to converged solution, the roofline of the planner kernel and the FP64
reference's throughput on this host's CPU; then, outside the timed steps, the
batched multi-query form against the plain per-query form, and the adjoint
refinement of a quadrotor path.
"""
import argparse
import itertools
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edges expanded/s; median ms to first & converged solution; batched vs plain"
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0


def flops_per_expansion(prob):
    """Algorithmic FLOPs of one candidate (add/sub/mul 1, FMA 2, div/sqrt/trig 1).

    Per RK4 step: 6d for the three stage updates, 6d for the final
    combination, four evaluations of f, the per-step validity arithmetic
    (speed norm 2P, boxes P each, spheres 3P each) and, for a path-length
    cost, 3P + 1.  Plus the edge cost, goal distance and heuristic once.
    The double integrators' RK4 step is the closed-form map it equals
    (p + h v + h^2/2 u, v + h u: three FMAs, 6 FLOP, per axis), so it is
    credited 6P, not the stage arithmetic.
    """
    from paper_2607_03987_amd import workloads as W
    d, P = prob.d, prob.npos
    f_eval = {W.DI2: 0, W.DI3: 0, W.CAR: 8, W.QUAD: 84, W.DUBINS: 8, W.UNI1: 4, W.UNI2: 4,
              W.ACROBOT: 38, W.CARTPOLE: 6}[prob.system]
    nb, ns = prob.box_c.shape[0], prob.sph_r.shape[0]
    speed = 2 * P if float(prob.vnorm_max) > 0 else 0
    rk4 = 6 * P if prob.system in (W.DI2, W.DI3) else 12 * d + 4 * f_eval
    step = rk4 + speed + P * nb + 3 * P * ns
    if prob.cost_kind == W.COST_PATH_LENGTH:
        step += 3 * P + 1
    return prob.T * step + 3 * P + 6


def nn_flops_per_pair(prob):
    return 3 * prob.d


PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_plan_di3_aox200ms_hbm_counters.md")
KERNEL_SOURCES = ["paper_2607_03987_amd/csrc/pakr.hip", "paper_2607_03987_amd/csrc/pakr_device.hpp",
                  "paper_2607_03987_amd/csrc/pakr_kernels.hpp", "include/pakr.h"]


def measured_traffic():
    """HBM bytes per planner launch from the committed rocprofv3 counter runs.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by the factors the
    same counters gave for a known-size copy; None once the kernel sources no
    longer hash to the profiled ones.
    """
    import hashlib
    try:
        txt = open(PMC_SUMMARY).read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        if ":" in line and line.split(":")[0] in ("fetch_factor", "write_factor",
                                                  "fetch_kib_per_dispatch",
                                                  "write_kib_per_dispatch", "source_sha256"):
            k, v = line.split(":", 1)
            vals[k] = v.split()[0]
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if vals.get("source_sha256") != h.hexdigest():
        return None
    return 1024.0 * (float(vals["fetch_kib_per_dispatch"]) * float(vals["fetch_factor"]) +
                     float(vals["write_kib_per_dispatch"]) * float(vals["write_factor"]))


VALU_SUMMARY = os.path.join(ROOT, "profiles", "k_plan_valu_counters.md")


def measured_valu(kernel: str):
    """Executed FP32 work of one kernel from the committed rocprofv3 counter runs.

    The summary holds, per kernel, lines `<kernel>.<field>: value` with
    executed_tflops (64 x SQ_INSTS_VALU_FLOPS_FP32, which counts the FLOPs of
    one wave instruction, over the dispatch time), valu_busy (SQ_ACTIVE_INST_VALU
    quad-cycles over the SIMDs' quad-cycles), active_lanes (SQ_THREAD_CYCLES_VALU
    / SQ_ACTIVE_INST_VALU, of 64) and flops_per_lane_inst; None once the kernel
    sources no longer hash to the profiled ones.
    """
    import hashlib
    try:
        txt = open(VALU_SUMMARY).read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        if ":" not in line or " " in line.split(":")[0]:
            continue
        k, v = line.split(":", 1)
        if v.split():
            vals[k] = v.split()[0]
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if vals.get("source_sha256") != h.hexdigest():
        return None
    out = {}
    for field in ("executed_tflops", "valu_busy", "active_lanes", "flops_per_lane_inst"):
        v = vals.get(f"{kernel}.{field}")
        if v is None:
            return None
        out[field] = float(v)
    out["executed_frac"] = out["executed_tflops"] / FP32_VECTOR_PEAK_TFLOPS
    out["source"] = "rocprofv3 --pmc counters, " + os.path.relpath(VALU_SUMMARY, ROOT)
    return out


def batched_vs_plain(torch, pakr, W, n_queries, rounds, iters_per_round, lanes=None,
                     settings=None):
    """The mixed batch (double integrator, car, quadrotor queries with uneven
    capacities) in one graph-launched persistent kernel, against the same
    queries planned one at a time with the whole GPU each.  Both forms run
    `rounds` AO-x rounds per query (deterministic), so per-query solution costs
    must be identical; the comparison is queries/s and solve latency."""
    probs = [p.replace(max_iters_per_round=iters_per_round)
             for p in W.config_c5(n_queries=n_queries, seed=0, settings=settings)]
    stream = torch.cuda.current_stream()
    # batched: one launch, replayed from a captured graph; lanes per candidate
    # per system from the tuned table
    lanes = lanes or {}
    bp = pakr.BatchPlan(probs, lanes=[lanes.get(p.system, 1) for p in probs])
    bp.graph_capture(max_rounds=rounds)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    bp.graph_launch()
    e1.record(stream)
    torch.cuda.synchronize()
    batch_wall = time.perf_counter() - t0
    batch_ms = e0.elapsed_time(e1)
    bst = [bp.status(q) for q in range(len(probs))]
    batch_flops = sum(s["expansions"] * flops_per_expansion(p) + s["nn_pairs"] * nn_flops_per_pair(p)
                      for s, p in zip(bst, probs))
    b_sols = [bp.solutions(q) for q in range(len(probs))]
    t_base = min(s["clock_start_ms"] for s in bst)
    b_done = [s["clock_end_ms"] - t_base for s in bst]
    b_first = [s["clock_start_ms"] - t_base + s["t_first_ms"] for s in bst if s["t_first_ms"] >= 0]
    # plain: the same queries one at a time, each with the whole GPU
    plans = [pakr.Plan(p) for p in probs]
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in plans]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, (a, b) in zip(plans, ev):
        a.record(stream)
        p.replan(max_rounds=rounds)
        b.record(stream)
    torch.cuda.synchronize()
    plain_wall = time.perf_counter() - t0
    p_ms = [a.elapsed_time(b) for a, b in ev]
    pst = [p.status() for p in plans]
    p_sols = [p.solutions() for p in plans]
    p_cum = list(itertools.accumulate(p_ms))
    p_first = [sum(p_ms[:q]) + s["t_first_ms"] for q, s in enumerate(pst) if s["t_first_ms"] >= 0]
    same = sum(1 for a, b in zip(b_sols, p_sols)
               if [(x["round"], x["iter"], x["node"], x["cost"]) for x in a] ==
               [(x["round"], x["iter"], x["node"], x["cost"]) for x in b])
    pct = lambda v, q: float(statistics.quantiles(v, n=100)[q - 1]) if len(v) >= 2 else None
    for p in plans:
        p.close()
    bp.close()
    return {
        "workload": f"{n_queries} mixed queries (3D double integrator / car / quadrotor, tree "
                    f"capacities log-uniform in [4096, 262144], 10-60 obstacles), "
                    f"{rounds} AO-x rounds each, at most {iters_per_round} iterations per round",
        "batched": {"queries_per_s": n_queries / (batch_ms / 1e3), "makespan_ms": batch_ms,
                    "wall_ms": batch_wall * 1e3, "grid": bst[0]["grid"],
                    "p50_done_ms": pct(b_done, 50), "p99_done_ms": pct(b_done, 99),
                    "p50_first_ms": pct(b_first, 50), "p99_first_ms": pct(b_first, 99),
                    "expansions": sum(s["expansions"] for s in bst),
                    "roofline": {"bound": "alu", "kernel": "k_batch",
                                 "achieved": batch_flops / (batch_ms / 1e3) / 1e12,
                                 "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                 "frac": batch_flops / (batch_ms / 1e3) / 1e12 /
                                 FP32_VECTOR_PEAK_TFLOPS,
                                 "executed": measured_valu("k_batch")}},
        "plain": {"queries_per_s": n_queries / (sum(p_ms) / 1e3), "total_ms": sum(p_ms),
                  "wall_ms": plain_wall * 1e3,
                  "p50_alone_ms": pct(p_ms, 50), "p99_alone_ms": pct(p_ms, 99),
                  "p50_queued_done_ms": pct(p_cum, 50), "p99_queued_done_ms": pct(p_cum, 99),
                  "p50_queued_first_ms": pct(p_first, 50), "p99_queued_first_ms": pct(p_first, 99),
                  "expansions": sum(s["expansions"] for s in pst)},
        "settings": {W.SYSTEM_NAMES[k]: v for k, v in (settings or {}).items()},
        "lanes": {W.SYSTEM_NAMES[k]: v for k, v in lanes.items()},
        "speedup_queries_per_s": sum(p_ms) / batch_ms,
        "queries_with_identical_solutions": f"{same}/{n_queries}",
        "solved": f"{sum(1 for x in b_sols if x)}/{n_queries}",
    }


def refinement_leg(torch, pakr, refine, W, budget_ms, n_multi):
    """Quadrotor workload: AO-x for `budget_ms`, then the adjoint refinement of
    the best path's controls (50 safeguarded Adam steps, each one forward and
    one adjoint rollout plus a trial rollout), and the planner's hard check.
    Also the throughput of the same refinement on n_multi paths at once
    (the found path with seeded control perturbations of 0.2% of the box)."""
    import numpy as np
    prob = W.config_c4(seed=0)
    plan = pakr.Plan(prob)
    plan.replan(budget_ms=budget_ms)
    st = plan.status()
    c4_flops = st["expansions"] * flops_per_expansion(prob) + st["nn_pairs"] * nn_flops_per_pair(prob)
    out = {"workload": "12D quadrotor AO-x, [0,10]^3, 50 spheres r U(0.3,1.2), B 8192, A 16, "
                       f"T 40, dt 0.02, tree capacity 2^20, {budget_ms:.0f} ms, then 50 adjoint "
                       "steps on the best path",
           "solved": st["n_solutions"] > 0, "c_best": st["c_best"],
           "planner": {"expansions_per_s": st["expansions"] / (st["call_ms"] / 1e3),
                       "time_to_first_ms": st["t_first_ms"], "grid": st["grid"],
                       "roofline": {"bound": "alu", "kernel": "k_plan<QUAD>",
                                    "achieved": c4_flops / (st["call_ms"] / 1e3) / 1e12,
                                    "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                    "frac": c4_flops / (st["call_ms"] / 1e3) / 1e12 /
                                    FP32_VECTOR_PEAK_TFLOPS}}}
    if st["n_solutions"] == 0:
        plan.close()
        return out
    states, actions, cost = plan.extract_path()
    plan.close()
    rs = W.refine_settings(prob)
    ref = refine.Refiner(prob, rs)
    stream = torch.cuda.current_stream()
    M = actions.shape[0]
    x0 = torch.from_numpy(states[:1].astype(np.float32)).cuda()
    U = torch.from_numpy(actions[None].astype(np.float32)).cuda()
    refine.refine_path(ref, x0, U, steps=2)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    res = refine.refine_path(ref, x0, U, steps=rs.steps, cost_bound=st["c_best"])
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    rng = np.random.default_rng(0)
    half = 0.5 * (np.asarray(prob.u_hi) - np.asarray(prob.u_lo))[:prob.m]
    Um = np.repeat(actions[None], n_multi, 0) + 0.002 * half * rng.uniform(-1, 1, (n_multi, M,
                                                                                  prob.m))
    Um = np.clip(Um, np.asarray(prob.u_lo)[:prob.m], np.asarray(prob.u_hi)[:prob.m])
    Um = torch.from_numpy(Um.astype(np.float32)).cuda()
    xm = x0.repeat(n_multi, 1)
    torch.cuda.synchronize()
    e0.record(stream)
    resm = refine.refine_path(ref, xm, Um, steps=rs.steps, cost_bound=st["c_best"])
    e1.record(stream)
    torch.cuda.synchronize()
    ms_multi = e0.elapsed_time(e1)
    ref.close()
    out.update({
        "edges": M, "rk4_steps_per_rollout": M * prob.T,
        "J_before": float(res["J_before"][0]), "J_after": float(res["J_after"][0]),
        "check_ok_bits": int(res["ok"][0]), "accepted": bool(res["accepted"][0]),
        "refine_ms": ms, "ms_per_adjoint_step": ms / rs.steps,
        "multi": {"paths": n_multi, "refine_ms": ms_multi,
                  "path_steps_per_s": n_multi * rs.steps / (ms_multi / 1e3),
                  "accepted": int(resm["accepted"].sum()),
                  "J_reduction_median": float((1 - resm["J_after"] / resm["J_before"])
                                              .median())},
    })
    return out


def other_systems_leg(torch, pakr, W, budget_ms, seeds):
    """The paper's other analytic systems (Dubins airplane, unicycles 1 and 2,
    acrobot and cart-pole swing-ups) at their default workloads: each seed is
    one single-query AO-x plan with a device-clock budget; expansions/s from the
    kernel's own event timing, the median time to the first solution, and the
    planner kernel's achieved FP32 rate against the vector peak."""
    out = {}
    stream = torch.cuda.current_stream()
    for name, mk in W.MORE_CONFIGS.items():
        w = pakr.Plan(mk(seed=10_000))
        w.replan(budget_ms=min(budget_ms, 20.0))
        torch.cuda.synchronize()
        w.close()
        exp = pairs = iters = 0
        ms, t_first = [], []
        steps = [0.0] * 6
        for sd in range(seeds):
            prob = mk(seed=sd)
            pl = pakr.Plan(prob)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            pl.replan(budget_ms=budget_ms)
            e1.record(stream)
            torch.cuda.synchronize()
            st, sols = pl.status(), pl.solutions()
            ms.append(e0.elapsed_time(e1))
            exp += st["expansions"]
            pairs += st["nn_pairs"]
            iters += st["total_iters"]
            steps = [a + b for a, b in zip(steps, st["step_ms"])]
            if sols:
                t_first.append(sols[0]["t_ms"])
            pl.close()
        prob = mk(seed=0)
        flops = exp * flops_per_expansion(prob) + pairs * nn_flops_per_pair(prob)
        tf = flops / (sum(ms) / 1e3) / 1e12
        out[name] = {"expansions_per_s": exp / (sum(ms) / 1e3),
                     "time_to_first_ms_median": statistics.median(t_first) if t_first else None,
                     "solved": f"{len(t_first)}/{seeds}", "B": prob.B, "A": prob.A, "T": prob.T,
                     "kernel_ms_mean": statistics.mean(ms),
                     "us_per_iteration": 1e3 * sum(ms) / max(iters, 1),
                     "step_us_per_iteration": step_split(steps, iters),
                     "roofline": {"bound": "alu", "achieved": tf,
                                  "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": tf / FP32_VECTOR_PEAK_TFLOPS}}
    return out


def saturating_rollout_leg(torch, pakr, W, iters, B=65536, A=16):
    """The rollout step at the largest batch one launch takes (B = 65536
    quadrotor candidates, 12D, T 40, 50 spheres): every iteration is capped at
    one per round, so each starts a new round from the root, the NN scan covers
    one node and the kernel time is the rollout, validity test and insertion of
    B candidates.  FP32 rate from the kernel's event timing, as for the planner
    legs."""
    prob = W.config_c4(B=B, A=A, n_cap=1 << 20, max_iters_per_round=1)
    stream = torch.cuda.current_stream()
    pl = pakr.Plan(prob)
    pl.expand(2)
    torch.cuda.synchronize()
    st0 = pl.status()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    pl.expand(iters)
    e1.record(stream)
    torch.cuda.synchronize()
    st = pl.status()
    ms = e0.elapsed_time(e1)
    exp = st["expansions"] - st0["expansions"]
    pairs = st["nn_pairs"] - st0["nn_pairs"]
    ins = st["insertions"] - st0["insertions"]
    flops = exp * flops_per_expansion(prob) + pairs * nn_flops_per_pair(prob)
    tf = flops / (ms / 1e3) / 1e12
    out = {"workload": f"12D quadrotor, [0,10]^3, 50 spheres r U(0.3,1.2), B {B}, A {A}, T 40, "
                       f"dt 0.02; one iteration per round, so every iteration expands the root",
           "iterations": iters, "kernel_ms": ms, "us_per_iteration": 1e3 * ms / iters,
           "expansions_per_s": exp / (ms / 1e3), "survival": ins / max(exp, 1),
           "grid": st["grid"], "step_ms": [round(v, 3) for v in st["step_ms"]],
           "roofline": {"bound": "alu", "kernel": "k_plan<QUAD>", "achieved": tf,
                        "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": tf / FP32_VECTOR_PEAK_TFLOPS,
                        "executed": measured_valu("k_plan_quad_b65536")}}
    pl.close()
    return out


def aox_leg(torch, pakr, make, seeds, budget_ms, lanes=0, wg_per_cu=0):
    """AO-x queries of one workload, one per seed (each its own scene and
    Philox key), each a single launch with a device-clock budget: the medians
    of Table 2's columns -- time to the first solution and its cost, time of
    the last improvement within the budget and the final cost -- over the
    solved seeds, the success rate, and expansions/s from the launches' own
    event timing."""
    stream = torch.cuda.current_stream()
    w = pakr.Plan(make(10_000), lanes=lanes, wg_per_cu=wg_per_cu)
    w.replan(budget_ms=min(budget_ms, 20.0))
    torch.cuda.synchronize()
    w.close()
    t1, c1, tf, cf, ms, exp, iters = [], [], [], [], [], 0, 0
    steps = [0.0] * 6
    for sd in seeds:
        prob = make(sd)
        pl = pakr.Plan(prob, lanes=lanes, wg_per_cu=wg_per_cu)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        pl.replan(budget_ms=budget_ms)
        e1.record(stream)
        torch.cuda.synchronize()
        st, sols = pl.status(), pl.solutions()
        ms.append(e0.elapsed_time(e1))
        exp += st["expansions"]
        iters += st["total_iters"]
        steps = [a + b for a, b in zip(steps, st["step_ms"])]
        if sols:
            t1.append(sols[0]["t_ms"])
            c1.append(sols[0]["cost"])
            tf.append(sols[-1]["t_ms"])
            cf.append(sols[-1]["cost"])
        pl.close()
    med = lambda v: statistics.median(v) if v else None
    prob = make(seeds[0])
    return {"workload": prob.name, "B": prob.B, "A": prob.A, "T": prob.T, "n_cap": prob.n_cap,
            "budget_ms": budget_ms, "seeds": f"{seeds[0]}..{seeds[-1]}",
            "solved": f"{len(t1)}/{len(seeds)}",
            "time_first_ms_median": med(t1), "cost_first_median": med(c1),
            "time_final_ms_median": med(tf), "cost_final_median": med(cf),
            "expansions_per_s": exp / (sum(ms) / 1e3),
            "us_per_iteration": 1e3 * sum(ms) / max(iters, 1),
            "step_us_per_iteration": step_split(steps, iters)}


STEP_NAMES = ["nn_scan", "barrier_a", "parent_reduce", "rollout", "barrier_b", "insert"]


def step_split(step_ms, iters):
    """Device time per iteration of each step of the loop (workgroup 0's clock)."""
    return {k: round(1e3 * v / max(iters, 1), 3) for k, v in zip(STEP_NAMES, step_ms)}


def host_cpu():
    """The host's CPU model, logical CPUs and the CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "usable": usable}


def _oracle_run(job):
    """Worker: `iters` iterations of the FP64 reference on workload c2, seed
    `seed`; returns its wall time and end state (run in a fresh process)."""
    seed, iters = job
    import oracle
    from paper_2607_03987_amd import workloads as W
    orc = oracle.OraclePlan(W.config_c2(seed=seed))
    t0 = time.perf_counter()
    for _ in range(iters):
        orc.iterate(report=False)
    dt = time.perf_counter() - t0
    st = orc.state()
    sols = [(s["round"], s["iter"], s["node"], s["cost"]) for s in orc.solutions()]
    return {"seed": seed, "seconds": dt, "expansions": st["expansions"], "n": st["n"],
            "n_solutions": st["n_solutions"], "solutions": sols}


def cpu_baseline(seconds, max_workers=16):
    """The FP64 reference on this host's cores, before the GPU is touched.

    One thread first runs workload c2 (seed 0) for about `seconds`; then one
    process per usable core (at most `max_workers`, the host share of one
    GPU) runs the same number of iterations on seeds 0, 1, ..., all at once.
    Worker 0 replays the single-thread run and must end in the same state
    (the reference is deterministic).  `value` is the all-core rate."""
    import multiprocessing as mp

    import oracle
    from paper_2607_03987_amd import workloads as W
    prob = W.config_c2(seed=0)
    orc = oracle.OraclePlan(prob)
    t0 = time.perf_counter()
    iters = 0
    while time.perf_counter() - t0 < seconds:
        orc.iterate(report=False)
        iters += 1
    dt1 = time.perf_counter() - t0
    st = orc.state()
    one = {"value": st["expansions"] / dt1, "iterations": iters, "seconds": dt1,
           "expansions": st["expansions"], "tree_nodes": st["n"],
           "solutions": st["n_solutions"]}
    host = host_cpu()
    workers = max(1, min(max_workers, host["usable"] or 1))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_run, [(sd, iters) for sd in range(workers)])
    wall = time.perf_counter() - t0
    r0 = res[0]
    same = (r0["expansions"] == st["expansions"] and r0["n"] == st["n"] and
            r0["solutions"] == [(s["round"], s["iter"], s["node"], s["cost"])
                                for s in orc.solutions()])
    total = sum(r["expansions"] for r in res)
    return {"value": total / wall, "unit": "expansions/s", "cores": workers, "kind": "oracle",
            "sample": f"{prob.name}: {workers} processes, seeds 0..{workers - 1}, {iters} "
                      f"iterations each ({total} expansions) in {wall:.1f} s wall, FP64; the "
                      f"single-thread run of seed 0 did the same {iters} iterations "
                      f"({st['expansions']} expansions, {st['n_solutions']} solution(s), tree "
                      f"{st['n']} nodes) in {dt1:.1f} s",
            "single_thread": one, "worker0_identical_to_single_thread": same,
            "host": host}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--budget-ms", type=float, default=200.0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--batch-queries", type=int, default=256)
    ap.add_argument("--batch-rounds", type=int, default=2)
    ap.add_argument("--batch-iters-per-round", type=int, default=50)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-refine", action="store_true")
    ap.add_argument("--no-other-systems", action="store_true")
    ap.add_argument("--other-systems-ms", type=float, default=100.0)
    ap.add_argument("--other-systems-seeds", type=int, default=3)
    ap.add_argument("--no-saturating-rollout", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the per-configuration AO-x legs (Table 2's columns)")
    ap.add_argument("--c1-seeds", type=int, default=100)
    ap.add_argument("--c1-budget-ms", type=float, default=50.0)
    ap.add_argument("--c2-seeds", type=int, default=100)
    ap.add_argument("--c3-seeds", type=int, default=100)
    ap.add_argument("--c3-budget-ms", type=float, default=200.0)
    ap.add_argument("--c4-seeds", type=int, default=100)
    ap.add_argument("--c4-budget-ms", type=float, default=500.0)
    ap.add_argument("--saturating-iters", type=int, default=50)
    ap.add_argument("--refine-budget-ms", type=float, default=500.0)
    ap.add_argument("--refine-paths", type=int, default=256)
    ap.add_argument("--maps-out", default="",
                    help="after the run (every plan closed, the device synchronized) write "
                         "/proc/self/maps to this file, to place the frames of any exit-time "
                         "fault")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before timing, run one plain device copy of this size (a known-size "
                         "kernel against which HBM counters are scaled)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the planner runs "
              "on a single GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    # the FP64 reference first, in fresh worker processes, before this
    # process touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_seconds)

    import torch

    from paper_2607_03987_amd import _build, autotune, pakr, refine, workloads as W

    if not os.path.exists(pakr.LIB_PATH):
        _build.build(force=True)
    torch.cuda.set_device(0)
    dev_name = torch.cuda.get_device_name(0)
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    tuned = autotune.load_table()
    lanes = args.lanes or int(tuned.get("single", {}).get("lanes", 0))
    wgpc = args.wg_per_cu or int(tuned.get("single", {}).get("workgroups_per_cu", 0))
    mk = lambda pr: pakr.Plan(pr, grid=args.grid, lanes=lanes, wg_per_cu=wgpc)
    warm = [mk(W.config_c2(seed=10_000 + i)) for i in range(args.warmup)]
    for p in warm:
        p.replan(budget_ms=args.budget_ms)
    torch.cuda.synchronize()
    for p in warm:
        p.close()

    probs = [W.config_c2(seed=s) for s in range(args.steps)]
    plans = [mk(pr) for pr in probs]
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in plans]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, (e0, e1) in zip(plans, ev):
        e0.record(stream)
        p.replan(budget_ms=args.budget_ms)
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    stats = [p.status() for p in plans]
    sols = [p.solutions() for p in plans]
    kernel_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    expansions = sum(s["expansions"] for s in stats)
    insertions = sum(s["insertions"] for s in stats)
    iters = sum(s["total_iters"] for s in stats)
    nn_pairs = sum(s["nn_pairs"] for s in stats)
    prob = probs[0]
    f_exp = flops_per_expansion(prob)
    f_nn = nn_flops_per_pair(prob)
    alg_flops = expansions * f_exp + nn_pairs * f_nn
    mean_kernel_s = statistics.mean(kernel_ms) / 1e3
    achieved_tflops = alg_flops / len(plans) / mean_kernel_s / 1e12
    nn_ms = sum(s["nn_ms"] for s in stats)
    roll_ms = sum(s["rollout_ms"] for s in stats)
    ins_ms = sum(s["insert_ms"] for s in stats)
    nn_bytes = nn_pairs / prob.K * prob.d * 4  # each iteration reads the tree once
    solved = [s for s in sols if s]
    t_first = [s[0]["t_ms"] for s in solved]
    t_conv = [s[-1]["t_ms"] for s in solved]
    c_first = [s[0]["cost"] for s in solved]
    c_final = [s[-1]["cost"] for s in solved]
    med = lambda v: statistics.median(v) if v else None

    out = {
        "metric": METRIC,
        "value": expansions / wall,
        "unit": "expansions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D double integrator AO-x: [0,10]^3, 30 random boxes side "
                               "U(0.5,2.5), start (1,1,1), goal ball (9,9,9) r 0.5, duration cost",
                   "B": prob.B, "A": prob.A, "K": prob.K, "T": prob.T, "dt": float(prob.dt),
                   "n_cap": prob.n_cap, "budget_ms": args.budget_ms,
                   "seeds": f"0..{args.steps - 1}", "grid": stats[0]["grid"],
                   "lanes_per_candidate": lanes or "auto", "device": dev_name},
        "time_to_first_ms_median": med(t_first),
        "time_to_converged_ms_median": med(t_conv),
        "cost_first_median": med(c_first),
        "cost_final_median": med(c_final),
        "solved": f"{len(solved)}/{len(plans)}",
        "iterations_per_step": iters / len(plans),
        "mean_tree_size": nn_pairs / max(iters, 1) / prob.K,
        "insertions_per_s": insertions / wall,
        "kernel_ms_mean": statistics.mean(kernel_ms),
        "phase_ms_per_step": {"nn": nn_ms / len(plans), "rollout": roll_ms / len(plans),
                              "insert": ins_ms / len(plans)},
        "step_ms_per_step": dict(zip(["nn_scan", "barrier_a", "parent_reduce", "rollout",
                                      "barrier_b", "insert"],
                                     [sum(s["step_ms"][i] for s in stats) / len(plans)
                                      for i in range(6)])),
        "nn_phase": {"tflops": nn_pairs * f_nn / (nn_ms / 1e3) / 1e12 if nn_ms else None,
                     "tree_read_gbs": nn_bytes / (nn_ms / 1e3) / 1e9 if nn_ms else None},
        "rollout_phase": {"tflops": expansions * f_exp / (roll_ms / 1e3) / 1e12 if roll_ms else None,
                          "flops_per_expansion": f_exp},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": measured_traffic(),
                     "executed": measured_valu("k_plan_di3"),
                     "kernel": "k_plan<DI3> (persistent AO-x planner), one launch per query"},
        "cpu_baseline": None,
        "batched": None,
        "refinement": None,
        "other_systems": None,
        "saturating_rollout": None,
        "configs": None,
    }
    for p in plans:
        p.close()
    if not args.no_batched:
        out["batched"] = batched_vs_plain(torch, pakr, W, args.batch_queries, args.batch_rounds,
                                          args.batch_iters_per_round,
                                          lanes=autotune.batch_lanes(tuned),
                                          settings=autotune.batch_settings(tuned))
    if not args.no_refine:
        out["refinement"] = refinement_leg(torch, pakr, refine, W, args.refine_budget_ms,
                                           args.refine_paths)
    if not args.no_other_systems:
        out["other_systems"] = other_systems_leg(torch, pakr, W, args.other_systems_ms,
                                                 args.other_systems_seeds)
    if not args.no_saturating_rollout:
        out["saturating_rollout"] = saturating_rollout_leg(torch, pakr, W, args.saturating_iters)
    if not args.no_configs:
        out["configs"] = {
            "c1": aox_leg(torch, pakr, lambda sd: W.config_c1(seed=sd), list(range(args.c1_seeds)),
                          args.c1_budget_ms),
            "c2": aox_leg(torch, pakr, lambda sd: W.config_c2(seed=sd), list(range(args.c2_seeds)),
                          args.budget_ms, lanes=lanes, wg_per_cu=wgpc),
            "c3": aox_leg(torch, pakr, lambda sd: W.config_c3(seed=sd), list(range(args.c3_seeds)),
                          args.c3_budget_ms),
            "c4": aox_leg(torch, pakr, lambda sd: W.config_c4(seed=sd), list(range(args.c4_seeds)),
                          args.c4_budget_ms),
        }
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    # every plan, batch and refiner above is closed; leave nothing queued on
    # the device for the interpreter's teardown
    import gc
    gc.collect()
    torch.cuda.synchronize()
    if args.maps_out:
        with open("/proc/self/maps") as src, open(args.maps_out, "w") as dst:
            dst.write(src.read())


if __name__ == "__main__":
    main()
