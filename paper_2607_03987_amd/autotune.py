"""Autotuner for the planner's launch and batch schedules.

Batched form: for each system of the mixed batch, a sample of that system's
queries is planned in one batched launch (teams sized automatically) for every
candidate (B, A, lanes) --
B and A on the grid shape of the paper's batch-size / branching-factor study
(Table 4), lanes = obstacle-test lanes per candidate.  Among the candidates
that solve at least 95% as many queries as the best one (first solution, one
round), the one with the most solved queries per second of makespan wins:
success first, then speed.  Single-query form: lanes per candidate and
workgroups per CU for the 3D double-integrator AO-x query, scored by
expansions per second.

The table is written to tuned.json next to this file; bench.py reads it.
Run: python -m paper_2607_03987_amd.autotune [--out PATH]   (needs a GPU)
"""
from __future__ import annotations

import json
import os
import time

from . import pakr, workloads as W

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")

B_GRID = (1024, 2048, 4096, 8192)
A_GRID = (4, 8, 16)
LANE_GRID = (1, 2, 4)


def load_table() -> dict:
    try:
        with open(TABLE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def batch_settings(table: dict | None = None) -> dict:
    """{system id: dict(B=..., A=...)} for workloads.config_c5."""
    table = load_table() if table is None else table
    out = {}
    for name, sid in (("di3", W.DI3), ("car", W.CAR), ("quad", W.QUAD)):
        ent = table.get("batch", {}).get(name)
        if ent:
            out[sid] = dict(B=int(ent["B"]), A=int(ent["A"]))
    return out


def batch_lanes(table: dict | None = None) -> dict:
    """{system id: lanes per candidate} for the batched form (1 where not tuned)."""
    table = load_table() if table is None else table
    out = {}
    for name, sid in (("di3", W.DI3), ("car", W.CAR), ("quad", W.QUAD)):
        ent = table.get("batch", {}).get(name)
        out[sid] = int(ent.get("lanes", 1)) if ent else 1
    return out


def _score_batch(torch, probs, lanes, iters_per_round):
    probs = [p.replace(max_iters_per_round=iters_per_round) for p in probs]
    bp = pakr.BatchPlan(probs, lanes=lanes)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    bp.replan(max_rounds=1)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    solved = sum(1 for q in range(len(probs)) if bp.status(q)["n_solutions"] > 0)
    bp.close()
    return solved / (ms / 1e3), solved, ms


def tune_batch(torch, n_per_system=48, iters_per_round=50, log=print) -> dict:
    res = {}
    for name, sid in (("di3", W.DI3), ("car", W.CAR), ("quad", W.QUAD)):
        runs = []
        for B in B_GRID:
            for A in A_GRID:
                for L in LANE_GRID:
                    probs = W.config_c5(n_queries=3 * n_per_system, seed=0,
                                        settings={sid: dict(B=B, A=A)})
                    probs = [p for p in probs if p.system == sid]
                    score, solved, ms = _score_batch(torch, probs, L, iters_per_round)
                    log(f"{name} B {B} A {A} lanes {L}: {solved}/{len(probs)} solved in "
                        f"{ms:.1f} ms -> {score:.1f} solved/s")
                    runs.append((score, B, A, L, solved, ms))
        top = max(r[4] for r in runs)
        best = max((r for r in runs if r[4] >= 0.95 * top), key=lambda r: r[0])
        res[name] = dict(B=best[1], A=best[2], lanes=best[3], solved=best[4], makespan_ms=best[5],
                         solved_per_s=best[0], sample=len(probs))
    return {"batch": res}


def tune_single(torch, budget_ms=200.0, seeds=(0, 1, 2, 3, 4, 5), log=print) -> dict:
    best = None
    for L in (2, 4, 8, 16):
        for k in (1, 2):
            exp, ms = 0, 0.0
            for sd in seeds:
                plan = pakr.Plan(W.config_c2(seed=sd), lanes=L, wg_per_cu=k)
                plan.replan(budget_ms=budget_ms)
                st = plan.status()
                exp += st["expansions"]
                ms += st["call_ms"]
                plan.close()
            rate = exp / (ms / 1e3)
            log(f"single c2 lanes {L} workgroups/CU {k}: {rate / 1e6:.1f} M expansions/s "
                f"over seeds {list(seeds)}")
            if best is None or rate > best[0]:
                best = (rate, L, k)
    return {"single": {"lanes": best[1], "workgroups_per_cu": best[2],
                       "expansions_per_s": best[0]}}


def main():
    import argparse

    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE, help="where to write the table")
    args = ap.parse_args()

    if not torch.cuda.is_available():
        raise SystemExit("the autotuner needs a GPU")
    t0 = time.time()
    table = {}
    table.update(tune_single(torch))
    table.update(tune_batch(torch))
    table["device"] = torch.cuda.get_device_name(0)
    table["seconds"] = round(time.time() - t0, 1)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps(table, indent=1), flush=True)


if __name__ == "__main__":
    main()
