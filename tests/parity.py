"""Step parity between the HIP planner and the FP64 reference.

For each GPU iteration the reference is re-seeded with the GPU's float32 tree
as it stood before the iteration (the snapshot is the first n0 slots of the
tree), recomputes the iteration in double precision, and adopts the GPU's
choice only where its own decision is a near tie (|margin| <= 1e-5, see the
reference's steering contract).  Then:

* targets and controls must be bit-identical (sampled values);
* parents, validity / prune / goal flags, insertion slots, the new node count
  and the goal candidate must be identical (no mismatch on a clear decision);
* final states and costs of valid candidates must agree within 1e-4 relative.
"""
import numpy as np

import oracle
from paper_2607_03987_amd import pakr

REL_TOL = 1e-4
# Refinement: dJ/dU of the float32 adjoint against the FP64 complex-step
# gradient (relative L2 norm of the difference), and the checkpointed states
# of a multi-edge rollout against the FP64 rollout (per component, relative to
# max(1, |x|), the planner's state tolerance).
GRAD_TOL = 1e-4
CKPT_TOL = 1e-4


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(1.0, np.abs(b))


def compare_iteration(prob, tr, rep, ctx=""):
    """Compare one decoded GPU trace record with the reference report."""
    B = prob.B
    np.testing.assert_array_equal(tr["targets"].view(np.uint32), rep.targets.view(np.uint32),
                                  err_msg=f"{ctx} targets")
    np.testing.assert_array_equal(tr["controls"].view(np.uint32), rep.controls.view(np.uint32),
                                  err_msg=f"{ctx} controls")
    assert rep.n_mismatch == 0, f"{ctx} {rep.n_mismatch} clear-cut decisions differ"
    np.testing.assert_array_equal(tr["parents"], rep.parents, err_msg=f"{ctx} parents")
    gv = (tr["flags"] & pakr.F_VALID) != 0
    ov = (rep.flags & oracle.F_VALID) != 0
    np.testing.assert_array_equal(gv, ov, err_msg=f"{ctx} valid flags")
    for gbit, obit, name in [(pakr.F_PRUNE_OK, oracle.F_PRUNE_OK, "prune"),
                             (pakr.F_GOAL, oracle.F_GOAL, "goal")]:
        np.testing.assert_array_equal(((tr["flags"] & gbit) != 0)[ov], ((rep.flags & obit) != 0)[ov],
                                      err_msg=f"{ctx} {name} flags")
    np.testing.assert_array_equal(tr["slots"], rep.slots, err_msg=f"{ctx} slots")
    assert tr["n1"] == rep.n1, f"{ctx} n1 {tr['n1']} vs {rep.n1}"
    assert tr["goal_j"] == rep.goal_j, f"{ctx} goal {tr['goal_j']} vs {rep.goal_j}"
    assert tr["end"] == rep.end, f"{ctx} end {tr['end']} vs {rep.end}"
    if ov.any():
        e = rel_err(tr["xnew"][ov], rep.xnew[ov]).max()
        assert e <= REL_TOL, f"{ctx} state rel err {e}"
        ec = rel_err(tr["cnew"][ov], rep.cnew[ov]).max()
        assert ec <= REL_TOL, f"{ctx} cost rel err {ec}"
    return dict(steered=rep.n_steered, valid=int(ov.sum()), kept=int((tr["slots"] >= 0).sum()),
                max_state_err=float(rel_err(tr["xnew"][ov], rep.xnew[ov]).max()) if ov.any() else 0.0)


def replay_records(prob, traces, orc, ctx=""):
    """Replay the records of a launch of many iterations in the reference.

    Before each iteration the reference is re-seeded with the GPU's float32
    tree as it stood then, rebuilt from the launch's own records (the root,
    then every earlier record's inserted candidates at their slots), exactly
    as step parity re-seeds it from a read-back of the tree.  A rollout is
    thus always compared from the same parent state: along a path of many
    edges the float32 and FP64 trees drift apart by the dynamics' own
    amplification of rounding error (chaotic systems such as the acrobot
    grow it past 1e-4 within a few edges), which says nothing about the
    kernel.
    """
    d, m, A = prob.d, prob.m, prob.A
    cap = prob.n_cap
    S = np.zeros((cap, d), np.float32)
    U = np.zeros((cap, m), np.float32)
    Pa = np.full(cap, -1, np.int32)
    C = np.zeros(cap, np.float32)
    S[0] = np.asarray(prob.x_init, np.float32)
    stats = []
    for i, tr in enumerate(traces):
        n0 = tr["n0"]
        c = tr["c_best_before"]
        orc.load_tree(S[:n0], U[:n0], Pa[:n0], C[:n0], tr["round"], tr["iter"],
                      c if np.isfinite(c) else np.inf)
        rep = orc.iterate(steer=dict(parents=tr["parents"], flags=tr["flags"],
                                     goal_j=tr["goal_j"]))
        stats.append(compare_iteration(prob, tr, rep, ctx=f"{ctx} iter {i} (round {tr['round']})"))
        js = np.nonzero(tr["slots"] >= 0)[0]
        sl = tr["slots"][js]
        assert sl.size == 0 or (sl.min() >= n0 and sl.max() < cap), (ctx, i)
        S[sl] = tr["xnew"][js]
        U[sl] = tr["controls"][js]
        Pa[sl] = tr["parents"][js // A]
        C[sl] = tr["cnew"][js]
    return stats


def step_parity(prob, n_iters, grid=0, log=None, lanes=0):
    """Run n_iters GPU iterations one at a time; replay each in the reference."""
    plan = pakr.Plan(prob, grid=grid, lanes=lanes)
    orc = oracle.OraclePlan(prob)
    stats = []
    c_best = float(prob.c0)
    for i in range(n_iters):
        st = plan.status()
        states, actions, parents, costs = plan.copy_tree()
        c_gpu = st["c_best"]
        orc.load_tree(states, actions, parents, costs, st["round"], st["iter"],
                      c_gpu if np.isfinite(c_gpu) else np.inf)
        tr = plan.expand(1, trace=True)[0]
        assert tr["round"] == st["round"] and tr["iter"] == st["iter"] and tr["n0"] == st["n_nodes"]
        rep = orc.iterate(steer=dict(parents=tr["parents"], flags=tr["flags"], goal_j=tr["goal_j"]))
        s = compare_iteration(prob, tr, rep, ctx=f"{prob.name} iter {i} (round {tr['round']})")
        stats.append(s)
        if log:
            log(f"iter {i}: n {tr['n0']}->{tr['n1']} valid {s['valid']} kept {s['kept']} "
                f"steered {s['steered']} err {s['max_state_err']:.2e} end {tr['end']}")
    plan.close()
    return stats
