"""The batched persistent kernel (k_batch) against the FP64 reference.

One launch plans a mixed batch -- every system, teams of one and of several
workgroups, different lanes per candidate, a ragged B, a query whose K = 1024
targets span two NN chunks, a finite initial cost bound -- and every query is
replayed, iteration by iteration, in the FP64 reference on the GPU's own
float32 tree (tests/parity.py): targets and controls bit for bit, parents,
flags, slots and the goal candidate exactly outside the near-tie band, states
and costs within 1e-4 relative.  Alg. 1 runs per query, so each query's
records are compared exactly as a single-query plan's are.
"""
import numpy as np
import pytest

import oracle
from paper_2607_03987_amd import pakr, workloads as W
from tests.parity import compare_iteration, replay_records

pytestmark = pytest.mark.gpu


def mixed_queries():
    cap = dict(n_cap=20000)
    return [
        # K = 1024 targets: two NN chunks of the batch kernel's 512-target staging
        W.config_c1(seed=2, B=2048, A=2, **cap),
        # ragged B (not a multiple of a rollout chunk), K = 100
        W.config_c2(seed=3, B=300, A=3, **cap),
        W.config_c3(seed=4, B=512, A=16, **cap),
        W.config_c4(seed=5, B=256, A=16, **cap),
        W.config_dubins(seed=6, B=512, A=8, **cap),
        W.config_uni1(seed=7, B=512, A=8, **cap),
        # a finite initial bound that splits the root's candidates (admissible h
        # is about 21.6 there and every 1 s edge adds 1): the prune decides
        # from the first iteration
        W.config_uni2(seed=8, B=512, A=8, c0=22.6, **cap),
        W.config_acrobot(seed=9, B=512, A=8, **cap),
        W.config_cartpole(seed=10, B=512, A=8, **cap),
    ]


TEAMS = [1, 3, 2, 1, 4, 1, 2, 3, 1]
LANES = [2, 16, 2, 1, 4, 8, 2, 1, 4]


def test_batch_kernel_step_parity_against_reference():
    probs = [p.replace(qid=q) for q, p in enumerate(mixed_queries())]
    bp = pakr.BatchPlan(probs, lanes=LANES, teams=TEAMS)
    assert [bp.team(q) for q in range(len(probs))] == TEAMS
    orcs = [oracle.OraclePlan(p) for p in probs]
    n_iters = 6
    totals = [dict(valid=0, kept=0, steered=0) for _ in probs]
    for i in range(n_iters):
        for q, (p, orc) in enumerate(zip(probs, orcs)):
            st = bp.status(q)
            states, actions, parents, costs = bp.copy_tree(q)
            c = st["c_best"]
            orc.load_tree(states, actions, parents, costs, st["round"], st["iter"],
                          c if np.isfinite(c) else np.inf)
        print(f"batch iteration {i}", flush=True)
        traces = bp.expand(1, trace=True)
        for q, (p, orc) in enumerate(zip(probs, orcs)):
            tr = traces[q][0]
            rep = orc.iterate(steer=dict(parents=tr["parents"], flags=tr["flags"],
                                         goal_j=tr["goal_j"]))
            s = compare_iteration(p, tr, rep, ctx=f"batch query {q} ({p.name}, team "
                                                  f"{TEAMS[q]}, lanes {LANES[q]}) iter {i}")
            for k in totals[q]:
                totals[q][k] += s[k]
    for q, t in enumerate(totals):
        print(f"  query {q} {probs[q].name}: {t}", flush=True)
        assert t["valid"] > 0, (q, probs[q].name)
    # the finite bound pruned something in the query that has one
    assert totals[6]["kept"] < totals[6]["valid"]
    bp.close()


def test_batch_expand_equals_replan_iterations():
    """pakr_batch_expand(n) and pakr_batch_replan(max_iters = n) run the same
    iterations, expanding in pieces equals one call, and the tiles that idle
    team members scan ahead (none or the automatic amount) change nothing."""
    probs = [p.replace(qid=q) for q, p in enumerate(mixed_queries()[:4])]
    a = pakr.BatchPlan(probs, lanes=LANES[:4], teams=TEAMS[:4], spec=-1)
    b = pakr.BatchPlan(probs, lanes=LANES[:4], teams=TEAMS[:4])
    a.expand(3)
    a.expand(4)
    b.replan(max_iters=7)
    for q in range(len(probs)):
        sa, sb = a.status(q), b.status(q)
        for key in ("total_iters", "insertions", "n_nodes", "round", "iter", "n_solutions"):
            assert sa[key] == sb[key], (q, key)
        for x, y in zip(a.copy_tree(q), b.copy_tree(q)):
            np.testing.assert_array_equal(x, y)
    a.close()
    b.close()


def test_batch_launch_of_many_iterations_against_reference():
    """A batch launch of many iterations (team members without a rollout chunk
    scan ahead), each query's records replayed in its own reference run,
    re-seeded every iteration with the tree the records rebuild."""
    probs = [p.replace(qid=q, max_iters_per_round=12) for q, p in enumerate(mixed_queries())]
    bp = pakr.BatchPlan(probs, lanes=LANES, teams=TEAMS)
    n_iters = 16
    traces = bp.expand(n_iters, trace=True)
    for q, p in enumerate(probs):
        print(f"query {q} {p.name}: {n_iters} iterations in one launch", flush=True)
        stats = replay_records(p, traces[q], oracle.OraclePlan(p),
                               ctx=f"batch launch query {q} ({p.name})")
        assert sum(s["valid"] for s in stats) > 0, (q, p.name)
    bp.close()
