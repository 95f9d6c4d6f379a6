"""HIP planner vs the FP64 reference (GPU tests).

Step parity (tests/parity.py) on every system at sizes the reference replays
in seconds -- several NN tiles, several rollout workgroups, ragged last tiles
-- plus the degenerate cases: K = 1, B not a multiple of 256, a tree that
fills up, an iteration cap, no obstacles, an explicit small grid.
"""
import numpy as np
import pytest

import oracle
from paper_2607_03987_amd import pakr, workloads as W
from tests.parity import compare_iteration, rel_err, replay_records, step_parity

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("cfg,kw,iters", [
    ("c1", {}, 40),
    ("c1", dict(seed=3, cost_kind=W.COST_DURATION), 30),
    ("c2", dict(B=1024, A=8, n_cap=40000), 12),
    ("c3", dict(B=1024, A=16, n_cap=40000), 12),
    ("c4", dict(B=512, A=16, n_cap=40000), 10),
])
def test_step_parity(cfg, kw, iters):
    prob = W.CONFIGS[cfg](**kw)
    print(f"case {prob.name} {kw}", flush=True)
    stats = step_parity(prob, iters, log=_log)
    assert sum(s["valid"] for s in stats) > 0


@pytest.mark.parametrize("cfg,kw,iters", [
    # the paper's own rule: c_new + ||pos(x_new) - x_goal|| < c_best (Alg. 1, Sec. IV)
    ("c1", dict(h_kind=W.H_PAPER_LITERAL, c0=14.0), 14),
    ("c2", dict(B=1024, A=8, n_cap=40000, h_kind=W.H_PAPER_LITERAL, c0=16.0), 8),
    # h = 0: the bound alone prunes (c_new < c_best)
    ("c1", dict(h_kind=W.H_NONE, c0=3.0), 14),
    ("c2", dict(B=1024, A=8, n_cap=40000, h_kind=W.H_NONE, c0=4.0), 8),
])
def test_step_parity_prune_rules(cfg, kw, iters):
    """Finite initial bounds under the literal heuristic and under h = 0: the
    prune flags must agree on every valid candidate, and the bound must both
    keep and reject candidates over the run."""
    prob = W.CONFIGS[cfg](**kw)
    print(f"case {prob.name} h_kind {prob.h_kind} c0 {prob.c0}", flush=True)
    stats = step_parity(prob, iters, log=_log)
    valid = sum(s["valid"] for s in stats)
    kept = sum(s["kept"] for s in stats)
    assert 0 < kept < valid, (kept, valid)


def _goal_ties(prob, tr):
    """Valid candidates of a record within 1e-5 of the goal radius (FP64 recount)."""
    valid = (tr["flags"] & pakr.F_VALID) != 0
    pos = tr["xnew"][:, :prob.npos].astype(np.float64)
    dist = np.linalg.norm(pos - np.asarray(prob.goal_c, np.float64)[:prob.npos], axis=1)
    return int((valid & (np.abs(dist - float(prob.goal_r)) <= 1e-5)).sum())


def _prune_ties(tr):
    """Valid candidates of a record within 1e-5 (relative) of the bound, h = 0."""
    valid = (tr["flags"] & pakr.F_VALID) != 0
    cb = tr["c_best_before"]
    if not np.isfinite(cb):
        return 0
    m = np.abs(tr["cnew"].astype(np.float64) - cb) / max(1.0, cb)
    return int((valid & (m <= 1e-5)).sum())


def test_near_tie_counters():
    """pakr_stats counts the candidates whose prune or goal decision lay within
    the near-tie band.  With h = 0 and the initial bound 5e-6 above one edge's
    duration, every valid child of the root is a prune near tie (cost = T dt,
    margin 5e-6 relative) and every deeper candidate is a whole edge away from
    the bound; both counts equal recounts from the iterations' records."""
    edge = float(np.float32(20) * np.float32(0.05))
    prob = W.config_c2(seed=3, B=512, A=8, n_cap=20000, h_kind=W.H_NONE, c0=edge + 5e-6)
    plan = pakr.Plan(prob)
    st0 = plan.status()
    assert st0["near_ties_prune"] == 0 and st0["near_ties_goal"] == 0
    tr = plan.expand(1, trace=True)[0]
    valid = int(((tr["flags"] & pakr.F_VALID) != 0).sum())
    st = plan.status()
    assert valid > 0 and _prune_ties(tr) == valid   # the construction holds
    assert st["near_ties_prune"] == valid, (st["near_ties_prune"], valid)
    assert st["near_ties_goal"] == _goal_ties(prob, tr)
    trs = plan.expand(3, trace=True)
    st2 = plan.status()
    assert st2["near_ties_prune"] == valid + sum(_prune_ties(t) for t in trs)
    assert st2["near_ties_goal"] == st["near_ties_goal"] + sum(_goal_ties(prob, t) for t in trs)
    plan.close()


@pytest.mark.parametrize("kw", [
    dict(B=300, A=3, n_cap=5000),          # ragged: B not a multiple of 256, K = 100
    dict(B=8, A=8, n_cap=2000),            # K = 1
    dict(B=256, A=1, n_cap=3000),          # A = 1
    dict(B=256, A=4, n_cap=300),           # the tree fills up
    dict(B=256, A=4, max_iters_per_round=3),  # iteration cap ends rounds
    dict(B=1, A=1, n_cap=2000),            # one candidate per iteration
    dict(T=1),                             # edges of a single RK4 step
])
def test_step_parity_edge_cases(kw):
    prob = W.config_c1(**kw)
    print(f"case c1 {kw}", flush=True)
    step_parity(prob, 12, log=_log)


def test_step_parity_start_inside_goal():
    # the goal test applies to new nodes (Alg. 1), so a start inside the goal
    # region ends the first rounds at their first iteration, each lowering the
    # bound; once no child can beat it, every candidate is pruned and the tree
    # stays at the root (no survivors at all)
    prob = W.config_c1(n_cap=4000)
    prob = prob.replace(goal_c=np.float32(prob.x_init[:2]))
    print("case c1 start inside goal", flush=True)
    step_parity(prob, 8, log=_log)
    ref = oracle.OraclePlan(prob)
    ends = [ref.iterate() for _ in range(8)]
    assert ends[0].goal_j >= 0 and ends[-1].n1 == 1  # the case covers both regimes


def test_step_parity_no_obstacles_and_small_grid():
    prob = W.config_c2(B=512, A=4, n_cap=20000)
    prob = prob.replace(box_c=prob.box_c[:0], box_h=prob.box_h[:0])
    print("case c2 no obstacles grid 8", flush=True)
    step_parity(prob, 8, grid=8, log=_log)


@pytest.mark.parametrize("grid", [1, 2, 3])
def test_step_parity_tiny_grids(grid):
    # one workgroup (no grid barrier at all), two (each owns every other tile),
    # three (ragged tile ownership); the NN key buffers alternate every iteration
    prob = W.config_c2(B=512, A=8, n_cap=20000)
    print(f"case c2 grid {grid}", flush=True)
    step_parity(prob, 7, grid=grid, log=_log)


def test_step_parity_targets_in_several_chunks():
    # K = 2048 targets: the NN scan stages them in LDS in two chunks of 1024
    prob = W.config_c1(B=4096, A=2, n_cap=20000)
    print("case c1 K 2048", flush=True)
    step_parity(prob, 5, log=_log)


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("cfg,kw", [("c2", dict(B=1024, A=8, n_cap=30000)),
                                    ("c4", dict(B=256, A=16, n_cap=30000))])
def test_step_parity_lanes_per_candidate(cfg, kw, lanes):
    prob = W.CONFIGS[cfg](**kw)
    print(f"case {prob.name} lanes {lanes}", flush=True)
    step_parity(prob, 6, lanes=lanes, log=_log)


@pytest.mark.parametrize("lanes", [16, 8])
def test_step_parity_ragged_sub_step_split(lanes):
    # T = 23 leaves the lanes of a double-integrator candidate unequal shares
    # of sub-steps and partly filled sweeps
    prob = W.config_c2(B=1024, A=8, n_cap=30000, T=23)
    print(f"case c2 T 23 lanes {lanes}", flush=True)
    step_parity(prob, 6, lanes=lanes, log=_log)


def test_expand_in_pieces_equals_one_call():
    prob = W.config_c1()
    a = pakr.Plan(prob)
    b = pakr.Plan(prob)
    ta = a.expand(20, trace=True)
    tb = b.expand(7, trace=True) + b.expand(13, trace=True)
    for x, y in zip(ta, tb):
        for key in ("parents", "slots", "flags"):
            np.testing.assert_array_equal(x[key], y[key])
        np.testing.assert_array_equal(x["xnew"].view(np.uint32), y["xnew"].view(np.uint32))
    sa, sb = a.copy_tree(), b.copy_tree()
    for x, y in zip(sa, sb):
        np.testing.assert_array_equal(x, y)


def test_replan_is_deterministic_and_launch_shape_independent():
    """Neither the grid size nor the lanes per candidate may change any result."""
    prob = W.config_c1(max_iters_per_round=80)
    res = []
    for grid, lanes in ((0, 0), (0, 0), (4, 1), (1, 1), (8, 8), (3, 2)):
        p = pakr.Plan(prob, grid=grid, lanes=lanes)
        p.replan(max_rounds=3)
        st = p.status()
        res.append((st["total_iters"], st["insertions"], [s["cost"] for s in p.solutions()],
                    p.copy_tree()))
        print(f"grid {grid} lanes {lanes}: {st['total_iters']} iters, {len(res[-1][2])} "
              f"solutions", flush=True)
    for r in res[1:]:
        assert r[0] == res[0][0] and r[1] == res[0][1] and r[2] == res[0][2]
        for x, y in zip(r[3], res[0][3]):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("cfg,kw", [("c2", dict(B=1024, A=8, n_cap=40000, max_iters_per_round=40)),
                                    ("c1", dict(T=23, max_iters_per_round=60))])
def test_double_integrator_lane_split_does_not_change_results(cfg, kw):
    """Double integrators split each edge's sub-steps and obstacles over the
    candidate's lanes in a way that depends on the lane count (and T): the
    trees must still be identical, bit for bit."""
    prob = W.CONFIGS[cfg](**kw)
    res = []
    for lanes in (1, 4, 16, 2):
        p = pakr.Plan(prob, lanes=lanes)
        p.replan(max_rounds=2)
        st = p.status()
        res.append((st["total_iters"], [s["cost"] for s in p.solutions()], p.copy_tree()))
        print(f"{prob.name} lanes {lanes}: {st['total_iters']} iters, {len(res[-1][1])} "
              f"solutions", flush=True)
        p.close()
    for r in res[1:]:
        assert r[0] == res[0][0] and r[1] == res[0][1]
        for x, y in zip(r[2], res[0][2]):
            np.testing.assert_array_equal(x, y)


def test_free_running_against_reference():
    """The reference runs its own FP64 tree, steered only on near ties."""
    prob = W.config_c1(seed=5, max_iters_per_round=60)
    plan = pakr.Plan(prob)
    orc = oracle.OraclePlan(prob)
    for i in range(80):
        tr = plan.expand(1, trace=True)[0]
        rep = orc.iterate(steer=dict(parents=tr["parents"], flags=tr["flags"], goal_j=tr["goal_j"]))
        compare_iteration(prob, tr, rep, ctx=f"free-running iter {i}")
    so, sg = orc.solutions(), plan.solutions()
    assert [(s["round"], s["iter"], s["node"]) for s in so] == \
           [(s["round"], s["iter"], s["node"]) for s in sg]
    if so:
        assert rel_err([s["cost"] for s in sg], [s["cost"] for s in so]).max() <= 1e-4


C1_LAUNCH = dict(seed=7, max_iters_per_round=45)


@pytest.mark.parametrize("cfg,kw,iters,tiers,cross", [
    ("c1", C1_LAUNCH, 90, dict(), 0),
    ("c1", C1_LAUNCH, 90, dict(tier0=256, tier1=-1), 1),
    ("c1", C1_LAUNCH, 90, dict(tier0=-1, tier1=-1), 0),
    # three tiers: 1 workgroup, then 8, then the grid, and back at each round
    ("c1", C1_LAUNCH, 90, dict(tier0=256, tier1=1024, tier1_grid=8), 2),
    ("c1", C1_LAUNCH, 90, dict(tier0=-1, tier1=2048, tier1_grid=32), 1),
    # the auto table with a small scan budget: 1, 32, 64, 128 workgroups, then the grid
    ("c1", C1_LAUNCH, 90, dict(tier0=128, tier_scan=120), 4),
    # ... and 8, 16, 32, 64, 128, then the grid
    ("c1", C1_LAUNCH, 90, dict(tier0=-1, tier1_grid=8, tier_scan=120), 5),
    ("c2", dict(seed=2, B=1024, A=8, n_cap=60000, max_iters_per_round=25), 40, dict(tier1=-1), 0),
    ("c2", dict(seed=2, B=1024, A=8, n_cap=60000, max_iters_per_round=25), 40,
     dict(tier1=4096, tier1_grid=64), 1),
    ("c2", dict(seed=2, B=1024, A=8, n_cap=60000, max_iters_per_round=25), 40,
     dict(tier_scan=1000), 2),
])
def test_one_launch_of_many_iterations_against_reference(cfg, kw, iters, tiers, cross):
    """All iterations in one launch: workgroups without a rollout chunk scan
    ahead for the next iteration and phase 1 skips what they covered, and the
    tiers of the tree (workgroup 0 alone, then sub-grids of growing size, then
    the grid) hand the loop over as the tree grows and take it back at every
    round; every iteration's record is replayed in the reference, re-seeded
    with the tree the records rebuild."""
    prob = W.CONFIGS[cfg](**kw)
    print(f"case {prob.name} one launch of {iters} iterations, tiers {tiers}", flush=True)
    plan = pakr.Plan(prob, **tiers)
    traces = plan.expand(iters, trace=True)
    replay_records(prob, traces, oracle.OraclePlan(prob), ctx=f"{prob.name} launch")
    rounds = {tr["round"] for tr in traces}
    sizes = [tr["n0"] for tr in traces]
    assert len(rounds) >= 2, "the run should cross a round end"
    st = plan.status()
    bounds = [b for b in st["tier_nodes"] if b > 0]
    assert len(bounds) >= cross, st["tier_nodes"]
    for bound in bounds[:cross]:
        # the tree grows across the tier's bound (and the round end takes it back)
        assert min(sizes) <= bound < max(sizes), (bound, max(sizes))
    plan.close()


def _auto_tiers(prob, G, g1, scan, tier0):
    """The auto table of sub-grid tiers, from its definition: grids doubling
    from g1 below the whole grid G, each taking the trees whose NN scan costs
    each of its workgroups at most `scan` cycles (K n (2d + 1) / 64 / grid),
    in whole tiles below the tree's capacity; empty bounds are dropped."""
    K = prob.B // prob.A
    out, prev, g = [], tier0, g1
    while g < G and len(out) < 6:
        lim = min(scan * g / (K * (2 * prob.d + 1) / 64), prob.n_cap)
        nk = int(lim)
        if nk < prob.n_cap:
            nk -= nk % 64
        if nk > prev:
            out.append((nk, g))
            prev = nk
            if nk >= prob.n_cap:
                break
        g *= 2
    return out


@pytest.mark.parametrize("cfg,kw,tiers", [
    ("c1", dict(), dict(tier1_grid=32)),
    ("c1", dict(), dict(tier0=-1, tier1_grid=8, tier_scan=120)),
    ("c1", dict(), dict(tier0=128, tier1_grid=32, tier_scan=120)),
    ("c2", dict(B=1024, A=8, n_cap=60000), dict(tier1_grid=32, tier_scan=1000)),
    ("c2", dict(), dict(tier1_grid=64)),
    ("uni1", dict(), dict(tier1_grid=32)),
    ("acrobot", dict(), dict(tier1_grid=64)),
    ("c1", dict(), dict(tier0=-1, tier1=3000, tier1_grid=16)),
])
def test_tier_table(cfg, kw, tiers):
    """The tier table a plan reports is the one its rule defines (first tier
    of one workgroup, then the sub-grid tiers, ascending)."""
    prob = (W.CONFIGS.get(cfg) or W.MORE_CONFIGS[cfg])(**kw)
    plan = pakr.Plan(prob, **tiers)
    st = plan.status()
    table = [(n, g) for n, g in zip(st["tier_nodes"], st["tier_grid"]) if n > 0]
    t0 = [e for e in table if e[1] == 1]
    tier0 = t0[0][0] if t0 else 0
    if tiers.get("tier0", 0) > 0:
        assert tier0 == tiers["tier0"]
    if tiers.get("tier1", 0) > 0:
        want = [(tiers["tier1"], tiers["tier1_grid"])]
    else:
        want = _auto_tiers(prob, st["grid"], tiers["tier1_grid"], tiers.get("tier_scan") or 10000,
                           tier0)
    print(f"{prob.name} grid {st['grid']} tiers {table}", flush=True)
    assert table == t0 + want
    assert all(a[0] < b[0] and a[1] < b[1] for a, b in zip(table, table[1:]))
    plan.close()


@pytest.mark.parametrize("cfg,kw,tiers", [
    ("c1", dict(max_iters_per_round=80),
     (dict(tier0=-1, tier1=-1), dict(tier0=256, tier1=-1), dict(tier0=1024, tier1=-1),
      dict(tier0=4096, tier1=-1), dict(), dict(tier0=1 << 20), dict(tier0=-1, tier1=1 << 20),
      dict(tier0=256, tier1=4096, tier1_grid=2), dict(tier0=1024, tier1=16384, tier1_grid=64),
      dict(tier_scan=120), dict(tier0=-1, tier1_grid=2, tier_scan=60))),
    # a first tier whose rollout takes several passes of workgroup 0, and a
    # second tier below the rollout workgroups of one batch
    ("c2", dict(B=1024, A=8, n_cap=60000, max_iters_per_round=40),
     (dict(tier0=-1, tier1=-1), dict(tier0=4096), dict(), dict(tier0=-1, tier1=16384, tier1_grid=4),
      dict(tier0=1024, tier1=16384, tier1_grid=96), dict(tier_scan=1000))),
])
def test_tiers_do_not_change_results(cfg, kw, tiers):
    """Where the tiers end and how many workgroups the second one has (none,
    4^4 .. 4^8 nodes, auto, always) changes no result."""
    prob = W.CONFIGS[cfg](**kw)
    res = []
    for t in tiers:
        p = pakr.Plan(prob, **t)
        p.replan(max_rounds=3)
        st = p.status()
        res.append((st["total_iters"], st["insertions"], st["nn_pairs"],
                    [(x["round"], x["iter"], x["node"], x["cost"]) for x in p.solutions()],
                    p.copy_tree()))
        print(f"{prob.name} tier0 {t}: {st['total_iters']} iterations, {len(res[-1][3])} "
              f"solutions", flush=True)
        p.close()
    for r in res[1:]:
        assert r[:4] == res[0][:4]
        for x, y in zip(r[4], res[0][4]):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("cfg,kw", [
    ("c1", dict(max_iters_per_round=80)),
    ("c2", dict(B=1024, A=8, n_cap=60000, max_iters_per_round=40)),
    ("c4", dict(B=512, A=16, n_cap=60000, max_iters_per_round=30)),
])
def test_scan_ahead_does_not_change_results(cfg, kw):
    """The tiles scanned ahead by idle workgroups (none, some, all) change no result."""
    prob = W.CONFIGS[cfg](**kw)
    res = []
    for spec in (-1, 1, 3, 0, 1024):
        p = pakr.Plan(prob, spec=spec)
        p.replan(max_rounds=3)
        st = p.status()
        res.append((st["total_iters"], st["insertions"], st["nn_pairs"],
                    [(x["round"], x["iter"], x["node"], x["cost"]) for x in p.solutions()],
                    p.copy_tree()))
        print(f"{prob.name} spec {spec}: {st['total_iters']} iterations, "
              f"{len(res[-1][3])} solutions", flush=True)
        p.close()
    for r in res[1:]:
        assert r[:4] == res[0][:4]
        for x, y in zip(r[4], res[0][4]):
            np.testing.assert_array_equal(x, y)


def test_extracted_path_is_feasible():
    prob = W.config_c1(max_iters_per_round=80)
    plan = pakr.Plan(prob)
    plan.replan(max_rounds=2)
    path = plan.extract_path()
    assert path is not None
    states, actions, cost = path
    assert np.array_equal(states[0], prob.x_init)
    cp = oracle.CProblem(prob)
    x = states[0].astype(float)
    total = 0.0
    for e in range(actions.shape[0]):
        ok, xT, c, amb = oracle.edge(cp, x, total, actions[e].astype(float))
        assert ok or amb
        assert rel_err(xT, states[e + 1]).max() <= 1e-4
        x, total = states[e + 1].astype(float), c
    assert np.linalg.norm(states[-1][:2] - prob.goal_c) <= prob.goal_r * (1 + 1e-6)
    assert abs(total - cost) <= 1e-4 * max(1.0, cost)
    sols = plan.solutions()
    assert sols[-1]["cost"] == pytest.approx(cost)
    assert all(b["cost"] < a["cost"] for a, b in zip(sols, sols[1:]))


@pytest.mark.parametrize("cfg,grid,tiers", [
    ("c2", 0, dict()), ("c2", 3, dict()), ("c2", 1, dict()),
    ("c2", 0, dict(tier1=16384, tier1_grid=64)),
    ("c1", 0, dict(tier0=1 << 20)), ("c1", 0, dict(tier0=1024, tier1=-1)), ("c1", 0, dict()),
    ("c1", 0, dict(tier0=256, tier1=4096, tier1_grid=16)), ("c1", 0, dict(tier0=-1, tier1=1 << 20)),
    ("c1", 0, dict(tier0=-1, tier1_grid=8, tier_scan=120)),
])
def test_budget_stop_ends_every_workgroup_at_one_iteration(cfg, grid, tiers):
    """Workgroup 0 takes the budget decision and every workgroup leaves at the
    same iteration -- also when only a tier's workgroups run while the others
    wait (c1: workgroup 0 alone or a sub-grid, always or in the small tiers
    of each round): the tree then equals that of a call capped at the same
    number of iterations, and planning resumes from it."""
    prob = (W.config_c2(B=512, A=8, n_cap=200000) if cfg == "c2"
            else W.config_c1(max_iters_per_round=60))
    print(f"case {cfg} budget 15 ms grid {grid} tiers {tiers}", flush=True)
    a = pakr.Plan(prob, grid=grid, **tiers)
    a.replan(budget_ms=15.0)
    st = a.status()
    assert st["status"] & pakr.S_BUDGET_EXPIRED, st["status"]
    assert st["call_iters"] > 0
    assert 15.0 <= st["call_ms"] <= 15.0 + 10.0, st["call_ms"]
    b = pakr.Plan(prob, grid=grid, **tiers)
    b.replan(max_iters=st["call_iters"])
    sb = b.status()
    assert sb["status"] & pakr.S_ITERS_DONE and not sb["status"] & pakr.S_BUDGET_EXPIRED
    for key in ("total_iters", "n_nodes", "round", "iter", "insertions", "n_solutions"):
        assert st[key] == sb[key], (key, st[key], sb[key])
    for x, y in zip(a.copy_tree(), b.copy_tree()):
        np.testing.assert_array_equal(x, y)
    ta = a.expand(4, trace=True)
    tb = b.expand(4, trace=True)
    for x, y in zip(ta, tb):
        for key in ("parents", "slots", "flags"):
            np.testing.assert_array_equal(x[key], y[key])
    a.close()
    b.close()
