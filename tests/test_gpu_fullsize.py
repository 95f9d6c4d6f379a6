"""Full-size parity at the launch configuration bench.py uses (GPU tests).

The configs' own B, A, T and tree capacities, with a goal ball too small to
reach so the tree grows to hundreds of thousands of nodes.  The reference
cannot replay whole iterations at this size, so sampled outputs are checked
one by one: target and control bits, the nearest neighbour of sampled targets
(FP64 brute force over the GPU's tree snapshot), sampled edges (validity,
final state, cost, prune flag), and properties that hold at any size
(survivors take consecutive slots in candidate order; parents precede
children).
"""
import numpy as np
import pytest

import oracle
from paper_2607_03987_amd import pakr, workloads as W
from tests.parity import rel_err, step_parity

pytestmark = pytest.mark.gpu


def _grow(plan, target, chunk):
    while True:
        st = plan.status()
        if st["n_nodes"] >= target:
            return st
        plan.expand(chunk)


@pytest.mark.parametrize("cfg,target,chunk", [("c2", 150000, 20), ("c3", 300000, 20),
                                              ("c4", 300000, 20)])
def test_sampled_parity_on_large_trees(cfg, target, chunk):
    prob = W.CONFIGS[cfg]().replace(goal_r=np.float32(1e-3))
    print(f"case {prob.name} full size, growing to {target} nodes", flush=True)
    plan = pakr.Plan(prob)
    st = _grow(plan, target, chunk)
    cp = oracle.CProblem(prob)
    rng = np.random.default_rng(0)
    for it in range(2):
        st = plan.status()
        states, actions, parents, costs = plan.copy_tree()
        n0 = states.shape[0]
        assert np.all(parents[1:] < np.arange(1, n0)) and parents[0] == -1
        tr = plan.expand(1, trace=True)[0]
        assert tr["n0"] == n0 and tr["round"] == st["round"] and tr["iter"] == st["iter"]
        print(f"iteration on a tree of {n0} nodes: {tr['survivors']} survivors", flush=True)
        # survivors take consecutive slots in candidate order
        keep = (tr["flags"] & pakr.F_KEEP) != 0
        ins = np.flatnonzero(tr["slots"] >= 0)
        np.testing.assert_array_equal(ins, np.flatnonzero(keep)[:ins.size])
        np.testing.assert_array_equal(tr["slots"][ins], n0 + np.arange(ins.size))
        assert tr["n1"] == n0 + ins.size
        # sampled targets: bits and nearest neighbour
        sdbl = states.astype(np.float64)
        for k in rng.choice(prob.K, size=12, replace=False):
            q = oracle.sample_state(cp, int(k), tr["iter"], tr["round"])
            np.testing.assert_array_equal(q.view(np.uint32), tr["targets"][k].view(np.uint32))
            best, d2, d2b = oracle.nearest(sdbl, q)
            g = int(tr["parents"][k])
            if g != best:
                dg = float(((q.astype(np.float64) - sdbl[g]) ** 2).sum())
                assert np.sqrt(dg) - np.sqrt(d2) <= 1e-5 * max(1.0, np.sqrt(d2)), (k, g, best)
        # sampled candidates: control bits and the edge itself
        for j in rng.choice(prob.B, size=48, replace=False):
            k, a = divmod(int(j), prob.A)
            u = oracle.sample_control(cp, k, a, tr["iter"], tr["round"])
            np.testing.assert_array_equal(u.view(np.uint32), tr["controls"][j].view(np.uint32))
            par = int(tr["parents"][k])
            ok, xT, c, amb = oracle.edge(cp, sdbl[par], float(costs[par]), u.astype(np.float64))
            gv = bool(tr["flags"][j] & pakr.F_VALID)
            assert gv == ok or amb, (j, gv, ok)
            if gv and ok:
                assert rel_err(tr["xnew"][j], xT).max() <= 1e-4
                assert rel_err(tr["cnew"][j], c).max() <= 1e-4
    plan.close()


def test_batched_form_at_bench_size_equals_single_query_plans():
    """The 256-query mixed batch in bench.py's launch configuration (tuned B and A per
    system, automatic team sizes, tuned lanes per system): sampled queries must end in
    the same state as planning them alone."""
    from paper_2607_03987_amd import autotune

    tuned = autotune.load_table()
    probs = [p.replace(max_iters_per_round=50)
             for p in W.config_c5(n_queries=256, seed=0, settings=autotune.batch_settings(tuned))]
    lanes = autotune.batch_lanes(tuned)
    print("case batch of 256 mixed queries, 2 rounds, auto teams", flush=True)
    bp = pakr.BatchPlan(probs, lanes=[lanes.get(p.system, 1) for p in probs])
    bp.replan(max_rounds=2)
    teams = [bp.team(q) for q in range(len(probs))]
    assert max(teams) > 1 and min(teams) >= 1
    rng = np.random.default_rng(3)
    sample = sorted(set(rng.choice(len(probs), 10, replace=False).tolist()) |
                    {int(np.argmax(teams))})
    for q in sample:
        single = pakr.Plan(probs[q], lanes=lanes.get(probs[q].system, 1))
        single.replan(max_rounds=2)
        sb, ss = bp.status(q), single.status()
        for key in ("total_iters", "expansions", "insertions", "n_nodes", "n_solutions"):
            assert sb[key] == ss[key], (q, teams[q], key, sb[key], ss[key])
        assert [(s["round"], s["iter"], s["node"], s["cost"]) for s in bp.solutions(q)] == \
               [(s["round"], s["iter"], s["node"], s["cost"]) for s in single.solutions()], q
        single.close()
    bp.close()


@pytest.mark.parametrize("one_iter_rounds", [True, False])
def test_step_parity_at_the_largest_batch(one_iter_rounds):
    """B = 65536, the largest batch one launch takes, on the quadrotor: every
    iteration replayed whole by the reference, from the root each time (the
    shape of bench.py's saturating-rollout measurement) or on the tree the
    first iteration grew."""
    kw = dict(B=65536, A=16, n_cap=1 << 20)
    if one_iter_rounds:
        kw["max_iters_per_round"] = 1
    prob = W.config_c4(**kw)
    print(f"case c4 B 65536 A 16 one-iteration rounds {one_iter_rounds}", flush=True)
    stats = step_parity(prob, 2, log=lambda m: print(m, flush=True))
    assert sum(s["valid"] for s in stats) > 0
