"""The record replay used by the one-launch parity tests, on the CPU.

A reference run stands in for the GPU: its per-iteration reports, rounded to
float32 like the GPU's trace records, are replayed by tests/parity.py's
replay_records in a second reference run, which must accept every record
and end with the same tree.  A record with a planted mistake (a wrong slot,
a wrong parent) must be rejected.
"""
import numpy as np
import pytest

import oracle
from paper_2607_03987_amd import workloads as W
from tests.parity import replay_records


def records_of(prob, n_iters):
    """Trace-shaped records of a free-running reference (float32 values)."""
    orc = oracle.OraclePlan(prob)
    recs = []
    for _ in range(n_iters):
        rep = orc.iterate()
        recs.append(dict(round=rep.round, iter=rep.iter, n0=rep.n0, n1=rep.n1,
                         goal_j=rep.goal_j, end=rep.end,
                         c_best_before=float(np.float32(rep.c_best_before)),
                         targets=rep.targets.copy(), parents=rep.parents.copy(),
                         controls=rep.controls.copy(),
                         xnew=rep.xnew.astype(np.float32), cnew=rep.cnew.astype(np.float32),
                         flags=rep.flags.copy(), slots=rep.slots.copy()))
    return recs, orc


def small_c1():
    return W.config_c1(seed=3, B=64, A=4, n_cap=2000, max_iters_per_round=20)


def test_replay_accepts_a_faithful_run_across_round_ends():
    prob = small_c1()
    recs, src = records_of(prob, 45)
    assert len({r["round"] for r in recs}) >= 2, "the run should cross a round end"
    dst = oracle.OraclePlan(prob)
    stats = replay_records(prob, recs, dst, ctx="cpu replay")
    assert sum(s["valid"] for s in stats) > 0
    a, b = src.tree(), dst.tree()
    assert a[0].shape == b[0].shape
    np.testing.assert_array_equal(a[2], b[2])        # parents
    np.testing.assert_allclose(a[0], b[0], rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("plant", ["slot", "parent"])
def test_replay_rejects_a_planted_mistake(plant):
    prob = small_c1()
    recs, _ = records_of(prob, 6)
    i = next(i for i, r in enumerate(recs) if (r["slots"] >= 0).sum() >= 2 and r["n0"] > 1)
    r = recs[i]
    if plant == "slot":
        js = np.nonzero(r["slots"] >= 0)[0]
        r["slots"][js[0]], r["slots"][js[1]] = r["slots"][js[1]], r["slots"][js[0]]
    else:
        r["parents"][0] = (r["parents"][0] + 1) % r["n0"]
    with pytest.raises(AssertionError):
        replay_records(prob, recs, oracle.OraclePlan(prob), ctx="planted")
