"""Batched multi-query planning (GPU tests).

One persistent launch plans many queries of mixed systems and uneven tree
capacities, each by a team of one or more workgroups.  Every query's results must be
bit-identical to planning it alone with the same parameters (the single-query
path is itself held to the FP64 reference by test_gpu_parity.py), and a
captured hipGraph of the launch must replay to the same state as direct calls.
"""
import numpy as np
import pytest

from paper_2607_03987_amd import pakr, workloads as W

pytestmark = pytest.mark.gpu

SMALL = {W.DI3: dict(B=512, A=8), W.CAR: dict(B=512, A=16), W.QUAD: dict(B=256, A=16)}


def small_batch(n, seed=0, iters_per_round=30):
    probs = W.config_c5(n_queries=n, seed=seed, settings=SMALL)
    return [p.replace(max_iters_per_round=iters_per_round, n_cap=min(p.n_cap, 30000))
            for p in probs]


TEAMS = {"single": 1, "auto": 0, "mixed": [1, 2, 3, 16, 1, 4, 2, 1, 5]}


@pytest.mark.parametrize("teams", list(TEAMS))
def test_batch_equals_single_query_plans(teams):
    probs = small_batch(9)
    print(f"case batch of 9 mixed queries, 2 rounds, teams {teams}", flush=True)
    bp = pakr.BatchPlan(probs, lanes=1, teams=TEAMS[teams])
    if teams == "mixed":
        assert [bp.team(q) for q in range(9)] == TEAMS["mixed"]
    bp.replan(max_rounds=2)
    for q, prob in enumerate(probs):
        pl = pakr.Plan(prob, lanes=1)
        pl.replan(max_rounds=2)
        sb, sp = bp.status(q), pl.status()
        for key in ("total_iters", "expansions", "insertions", "n_nodes", "round", "iter",
                    "n_solutions", "nn_pairs"):
            assert sb[key] == sp[key], (q, key, sb[key], sp[key])
        assert sb["c_best"] == sp["c_best"] or (np.isinf(sb["c_best"]) and np.isinf(sp["c_best"]))
        assert [(s["round"], s["iter"], s["node"], s["cost"]) for s in bp.solutions(q)] == \
               [(s["round"], s["iter"], s["node"], s["cost"]) for s in pl.solutions()]
        a, b = bp.extract_path(q), pl.extract_path()
        assert (a is None) == (b is None)
        if a is not None:
            np.testing.assert_array_equal(a[0], b[0])
            np.testing.assert_array_equal(a[1], b[1])
        pl.close()
    bp.close()


@pytest.mark.parametrize("lanes", [2, 8])
def test_batch_lane_count_does_not_change_results(lanes):
    probs = small_batch(6, seed=1)
    print(f"case batch lanes {lanes}", flush=True)
    a = pakr.BatchPlan(probs, lanes=1)
    b = pakr.BatchPlan(probs, lanes=lanes)
    a.replan(max_iters=12)
    b.replan(max_iters=12)
    for q in range(len(probs)):
        sa, sb = a.status(q), b.status(q)
        assert (sa["insertions"], sa["n_nodes"], sa["round"]) == \
               (sb["insertions"], sb["n_nodes"], sb["round"]), q
        assert a.solutions(q) and b.solutions(q) or not (a.solutions(q) or b.solutions(q))


def test_graph_replays_match_direct_calls():
    probs = small_batch(6, seed=2)
    print("case graph replay x3 of 4 iterations", flush=True)
    bg = pakr.BatchPlan(probs, lanes=1)
    bd = pakr.BatchPlan(probs, lanes=1)
    bg.graph_capture(max_iters=4)
    torch = bg.torch
    for rep in range(3):
        bg.graph_launch()
        bd.replan(max_iters=4)
        # eager work and a synchronisation between replays
        x = torch.arange(1000, device="cuda", dtype=torch.float32)
        assert float((x * 2).sum().item()) == 999000.0
        torch.cuda.synchronize()
        for q in range(len(probs)):
            sg, sd = bg.status(q), bd.status(q)
            assert sg["total_iters"] == 4 * (rep + 1) == sd["total_iters"], (rep, q)
            for key in ("insertions", "n_nodes", "round", "iter", "n_solutions", "nn_pairs"):
                assert sg[key] == sd[key], (rep, q, key)
            assert bg.solutions(q) == [dict(s, t_ms=t["t_ms"]) for s, t in
                                       zip(bd.solutions(q), bg.solutions(q))]
