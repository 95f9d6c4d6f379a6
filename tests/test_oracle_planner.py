"""Pins for the reference planner loop (Alg. 1 and the AO-x outer loop).

* brute-force agreement with a second naive transcription (tests/pyplanner.py)
  on tiny double-integrator problems;
* tree invariants after every iteration: the root, parent[i] < i, the stored
  state / cost equal a fresh rollout from the parent, survivors pass the bound
  that was in force;
* AO-x: solution costs strictly decrease, every extracted path re-simulated
  from x_init stays valid and ends in the goal, h never exceeds the remaining
  cost along a solution path (admissibility);
* Sec. IV-B: with A > 1 the candidate set of the first batch contains every
  candidate of the A = 1 planner with the same K;
* capacity / iteration-cap round endings and the steering contract.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2607_03987_amd import workloads as W
from tests.pyplanner import PyPlanner


def tiny_di2(seed, **kw):
    args = dict(B=16, A=4, T=5, n_cap=300, max_iters_per_round=40)
    args.update(kw)
    return W.config_c1(seed=seed, **args)


@pytest.mark.parametrize("seed,cost_kind", [(0, W.COST_PATH_LENGTH), (1, W.COST_DURATION),
                                            (2, W.COST_PATH_LENGTH), (3, W.COST_DURATION)])
def test_matches_naive_transcription(seed, cost_kind):
    p = tiny_di2(seed, cost_kind=cost_kind, dt=np.float32(0.1))
    orc = oracle.OraclePlan(p)
    ref = PyPlanner(p)
    for it in range(120):
        rep = orc.iterate()
        ref.step()
        st = orc.state()
        assert st["round"] == ref.round and st["iter"] == ref.iter
        assert st["n"] == len(ref.X)
        states, actions, parents, costs = orc.tree()
        np.testing.assert_allclose(states, np.array(ref.X), rtol=0, atol=1e-12)
        np.testing.assert_array_equal(parents, np.array(ref.P))
        np.testing.assert_allclose(costs, np.array(ref.C), rtol=1e-13, atol=1e-13)
        np.testing.assert_array_equal(actions, np.array(ref.U))
    sols = orc.solutions()
    assert [(s["round"], s["iter"], s["node"]) for s in sols] == [s[:3] for s in ref.solutions]
    np.testing.assert_allclose([s["cost"] for s in sols], [s[3] for s in ref.solutions], rtol=1e-13)


def _check_tree(orc, p, rep):
    cp = orc.cp
    states, actions, parents, costs = orc.tree()
    n = states.shape[0]
    assert parents[0] == -1 and costs[0] == 0.0
    np.testing.assert_array_equal(states[0], p.x_init.astype(float))
    assert np.all(parents[1:] >= 0) and np.all(parents[1:] < np.arange(1, n))
    for i in range(max(1, rep.n0), rep.n1 if rep.end == oracle.END_NONE else 0):
        ok, xT, c, _ = oracle.edge(cp, states[parents[i]], costs[parents[i]], actions[i])
        assert ok
        np.testing.assert_array_equal(xT, states[i])
        assert c == costs[i]
        assert c + oracle.heuristic(cp, xT) < rep.c_best_before


@pytest.mark.parametrize("cfg,kw", [
    ("c1", {}),
    ("c2", dict(B=512, A=8, n_cap=20000)),
    ("c3", dict(B=512, A=16, n_cap=20000)),
    ("c4", dict(B=256, A=16, n_cap=20000)),
])
def test_tree_invariants_every_iteration(cfg, kw):
    p = W.CONFIGS[cfg](**kw)
    orc = oracle.OraclePlan(p)
    iters = 25 if cfg != "c1" else 60
    for _ in range(iters):
        rep = orc.iterate()
        # slots are consecutive at the frontier, in candidate order
        ins = np.flatnonzero(rep.flags & oracle.F_INSERTED)
        np.testing.assert_array_equal(rep.slots[ins], rep.n0 + np.arange(ins.size))
        keep = np.flatnonzero(rep.flags & oracle.F_KEEP)
        assert ins.size == min(keep.size, p.n_cap - rep.n0)
        np.testing.assert_array_equal(ins, keep[:ins.size])
        if math.isinf(rep.c_best_before):
            assert np.all((rep.flags & oracle.F_PRUNE_OK) != 0)   # no bound yet: no prune
        if rep.end == oracle.END_NONE:
            _check_tree(orc, p, rep)
        if rep.goal_j >= 0:
            g = np.flatnonzero(((rep.flags & oracle.F_INSERTED) != 0) & ((rep.flags & oracle.F_GOAL) != 0))
            assert rep.goal_j == g[np.argmin(rep.cnew[g])]
            assert rep.c_best_after == rep.cnew[rep.goal_j] < rep.c_best_before


def _resimulate(p, states, actions):
    """Re-run an extracted path from x_init with a test-side RK4 (double integrators)."""
    D, h = p.npos, float(p.dt)
    x = p.x_init.astype(float)
    length = 0.0
    for e in range(actions.shape[0]):
        u = actions[e]
        for _ in range(p.T):
            k1 = np.concatenate([x[D:], u])
            k2 = np.concatenate([x[D:] + h / 2 * k1[D:], u])
            k3 = np.concatenate([x[D:] + h / 2 * k2[D:], u])
            k4 = np.concatenate([x[D:] + h * k3[D:], u])
            xn = x + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
            length += float(np.linalg.norm(xn[:D] - x[:D]))
            pos = xn[:D]
            assert np.all(pos >= p.ws_lo) and np.all(pos <= p.ws_hi)
            assert np.linalg.norm(xn[D:]) <= p.vnorm_max + 1e-12
            for c, hh in zip(p.box_c.astype(float), p.box_h.astype(float)):
                assert np.any(np.abs(pos - c) > hh)
            x = xn
        np.testing.assert_allclose(x, states[e + 1], atol=1e-9)
    cost = length if p.cost_kind == W.COST_PATH_LENGTH else actions.shape[0] * p.T * h
    return x, cost


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_aox_solutions_improve_and_paths_are_feasible(seed):
    p = W.config_c1(seed=seed, max_iters_per_round=60)
    orc = oracle.OraclePlan(p)
    costs = []
    for _ in range(400):
        rep = orc.iterate()
        if rep.end == oracle.END_GOAL:
            path = orc.best_path()
            assert path is not None
            states, actions, cost = path
            assert cost == rep.c_best_after
            xT, c_sim = _resimulate(p, states, actions)
            assert np.linalg.norm(xT[:2] - p.goal_c) <= p.goal_r + 1e-9
            assert c_sim == pytest.approx(cost, rel=1e-9)
            # admissible heuristic: h(node) <= cost remaining along the path
            cp = orc.cp
            seg = np.cumsum([0.0] + [np.linalg.norm(states[i + 1, :2] - states[i, :2])
                                     for i in range(states.shape[0] - 1)])
            for i in range(states.shape[0]):
                assert oracle.heuristic(cp, states[i]) <= cost - seg[i] + 1e-9
            costs.append(cost)
    assert len(costs) >= 1
    assert all(b < a for a, b in zip(costs, costs[1:]))
    assert [s["cost"] for s in orc.solutions()] == costs


def test_branching_superset_of_single_control():
    """Sec. IV-B: the A>1 planner evaluates every candidate the A=1 planner does."""
    p1 = W.config_c2(B=256, A=1, n_cap=5000)
    p8 = W.config_c2(B=256 * 8, A=8, n_cap=5000)
    r1 = oracle.OraclePlan(p1).iterate()
    r8 = oracle.OraclePlan(p8).iterate()
    np.testing.assert_array_equal(r1.targets, r8.targets)
    np.testing.assert_array_equal(r1.parents, r8.parents)
    np.testing.assert_array_equal(r1.controls, r8.controls[0::8])
    np.testing.assert_array_equal(r1.xnew, r8.xnew[0::8])
    np.testing.assert_array_equal(r1.flags & oracle.F_KEEP, r8.flags[0::8] & oracle.F_KEEP)


def test_tree_full_ends_round_and_keeps_bound():
    p = W.config_c1(n_cap=40, B=64, A=4)
    orc = oracle.OraclePlan(p)
    rep = orc.iterate()
    assert rep.n1 == 40 and rep.end == oracle.END_TREE_FULL
    assert ((rep.flags & oracle.F_INSERTED) != 0).sum() == 39
    st = orc.state()
    assert st["round"] == 1 and st["n"] == 1 and st["iter"] == 0 and math.isinf(st["c_best"])


def test_iteration_cap_ends_round():
    p = W.config_c1(max_iters_per_round=3)
    orc = oracle.OraclePlan(p)
    ends = [orc.iterate().end for _ in range(4)]
    assert ends[:3] == [0, 0, oracle.END_ITER_CAP]
    assert orc.state()["round"] == 1 and orc.state()["iter"] == 1


def test_steering_contract():
    p = W.config_c1()
    a = oracle.OraclePlan(p)
    for _ in range(5):
        a.iterate()
    b = oracle.OraclePlan(p)
    for _ in range(5):
        b.iterate()
    ref = a.iterate()
    # steering with the same decisions changes nothing
    same = b.iterate(steer=dict(parents=ref.parents, flags=ref.flags, goal_j=ref.goal_j))
    assert same.n_mismatch == 0 and same.n_steered == 0
    np.testing.assert_array_equal(same.slots, ref.slots)
    # a flipped clear-cut validity decision is a mismatch and is not adopted
    c = oracle.OraclePlan(p)
    for _ in range(5):
        c.iterate()
    j = int(np.flatnonzero((ref.flags & oracle.F_VALID) & (ref.amb == 0))[0])
    fl = ref.flags.copy()
    fl[j] ^= oracle.F_VALID
    par = ref.parents.copy()
    k = int(np.flatnonzero(ref.nn_tie == 0)[0])
    par[k] = (par[k] + 1) % max(ref.n0, 2)
    bad = c.iterate(steer=dict(parents=par, flags=fl, goal_j=ref.goal_j))
    assert bad.n_mismatch >= 2 and bad.n_steered == 0
    np.testing.assert_array_equal(bad.flags, ref.flags)
