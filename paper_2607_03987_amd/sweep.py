"""Batch-size x branching-factor study on the quadrotor workload.

The grid shape of the paper's sensitivity study (Table 4, Sec. V-D): batch
sizes B in {4096, 8192, 16384, 32768} and branching factors A in
{2, 16, 64, 128}, with the 12D quadrotor among 50 random spheres.  For every
cell, `trials` seeded scenes are planned until the first solution (one AO-x
round) or the time limit, and the cell reports the success rate and, over the
solved trials, the median time to the first solution, the iterations it took
and the tree size when it was found.

Run: python -m paper_2607_03987_amd.sweep [--trials N] [--limit-ms MS] [--out PATH]
[--md PATH] (needs a GPU).  Prints one JSON object and writes it to --out if
given; --md writes the table in the paper's layout with the command and the
SHA-256 of the kernel sources it ran.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

from . import pakr, workloads as W

B_GRID = (4096, 8192, 16384, 32768)
A_GRID = (2, 16, 64, 128)


def run_cell(B: int, A: int, trials: int, limit_ms: float, seed0: int = 0) -> dict:
    solved, t_first, iters, nodes = 0, [], [], []
    for s in range(seed0, seed0 + trials):
        prob = W.config_c4(seed=s, B=B, A=A)
        plan = pakr.Plan(prob)
        plan.replan(budget_ms=limit_ms, max_rounds=1)
        sols = plan.solutions()
        if sols:
            solved += 1
            first = sols[0]
            t_first.append(first["t_ms"])
            iters.append(first["iter"] + 1)
            nodes.append(first["n_nodes"])
        plan.close()
    med = lambda v: statistics.median(v) if v else None
    return {"B": B, "A": A, "trials": trials, "success_pct": 100.0 * solved / trials,
            "time_ms": med(t_first), "iters": med(iters), "nodes": med(nodes)}


_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_2607_03987_amd/csrc/pakr.hip", "paper_2607_03987_amd/csrc/pakr_device.hpp",
                  "paper_2607_03987_amd/csrc/pakr_kernels.hpp", "include/pakr.h"]


def source_sha256() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(_ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def markdown(out: dict, command: str) -> str:
    """The study as a table shaped like the paper's (rows: B and metric, columns: A)."""
    cells = {(c["B"], c["A"]): c for c in out["cells"]}
    As = sorted({a for _, a in cells})
    Bs = sorted({b for b, _ in cells})
    fmt = lambda v, f: "-" if v is None else f.format(v)
    lines = [f"# Batch size x branching factor on the quadrotor ({out['trials_per_cell']} trials "
             f"per cell)", "",
             out["workload"] + ".", "",
             f"Command: `{command}`", "",
             f"Device: {out['device']}; {out['seconds']} s; kernel sources sha256 "
             f"{out.get('source_sha256', '?')}.", "",
             "Medians over the solved trials of each cell (time to the first solution, the "
             "iterations it took, the tree size then).", "",
             "| B | metric | " + " | ".join(f"A = {a}" for a in As) + " |",
             "|---|---|" + "---|" * len(As)]
    for B in Bs:
        for key, name, f in (("success_pct", "success %", "{:.0f}"), ("time_ms", "time ms", "{:.1f}"),
                             ("iters", "iters", "{:.0f}"), ("nodes", "nodes", "{:.0f}")):
            row = [fmt(cells[(B, a)][key], f) if (B, a) in cells else "-" for a in As]
            lines.append(f"| {B} | {name} | " + " | ".join(row) + " |")
    return "\n".join(lines) + "\n"


def main():
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--trials", type=int, default=20)
    ap.add_argument("--limit-ms", type=float, default=1000.0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--md", default=None)
    args = ap.parse_args()
    if not torch.cuda.is_available():
        raise SystemExit("the sweep needs a GPU")
    torch.cuda.set_device(0)
    t0 = time.time()
    cells = []
    for B in B_GRID:
        for A in A_GRID:
            cell = run_cell(B, A, args.trials, args.limit_ms)
            print(json.dumps(cell), flush=True)
            cells.append(cell)
    out = {"workload": "12D quadrotor, [0,10]^3, 50 spheres r U(0.3,1.2), start (1,1,1), goal "
                       "ball (9,9,9) r 1, T 40, dt 0.02, tree capacity 2^20; one AO-x round "
                       "(first solution) per trial",
           "trials_per_cell": args.trials, "limit_ms": args.limit_ms,
           "device": torch.cuda.get_device_name(0), "seconds": round(time.time() - t0, 1),
           "source_sha256": source_sha256(), "cells": cells}
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
    if args.md:
        with open(args.md, "w") as f:
            f.write(markdown(out, "python -m paper_2607_03987_amd.sweep " + " ".join(sys.argv[1:])))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
