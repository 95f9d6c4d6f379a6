"""Failure handling on the GPU, forced from the host.

A grid-barrier wait limit of a few nanoseconds (pakr_set_barrier_timeout)
makes the first barrier that any workgroup has to wait at fail; every wait in
the kernels is bounded, so each workgroup leaves through that path and the
launch completes normally.  The failure must then be reported: status and the
read-back calls return PAKR_E_DEVICE, and the plan or batch refuses later
launches.  Nothing here faults or hangs the GPU.
"""
import pytest

from paper_2607_03987_amd import pakr, workloads as W

pytestmark = pytest.mark.gpu

E_DEVICE = -8


@pytest.fixture
def tiny_barrier_timeout():
    pakr.set_barrier_timeout(1e-6)
    yield
    pakr.set_barrier_timeout(0.0)


def test_single_plan_reports_barrier_timeout(tiny_barrier_timeout):
    prob = W.config_c2(B=512, A=8, n_cap=20000)
    plan = pakr.Plan(prob)          # one workgroup per CU: every iteration has two grid barriers
    print("case c2 single plan, barrier timeout 1e-6 ms", flush=True)
    plan.replan(max_iters=40)
    with pytest.raises(pakr.PakrError) as ei:
        plan.status()
    assert ei.value.code == E_DEVICE
    with pytest.raises(pakr.PakrError) as ei:
        plan.replan(max_iters=1)
    assert ei.value.code == E_DEVICE
    plan.close()


def test_batch_reports_barrier_timeout(tiny_barrier_timeout):
    probs = [p.replace(max_iters_per_round=10, n_cap=min(p.n_cap, 20000))
             for p in W.config_c5(n_queries=4, seed=3,
                                  settings={W.DI3: dict(B=512, A=8), W.CAR: dict(B=512, A=16),
                                            W.QUAD: dict(B=256, A=16)})]
    bp = pakr.BatchPlan(probs, lanes=1, teams=[4, 2, 3, 1])
    print("case batch of 4, teams 4/2/3/1, barrier timeout 1e-6 ms", flush=True)
    bp.replan(max_iters=20)
    codes = []
    for q in range(len(probs)):
        try:
            bp.status(q)
            codes.append(0)
        except pakr.PakrError as e:
            codes.append(e.code)
    # query 3 plans alone (no grid barrier); the others have teams and fail
    assert codes[0] == E_DEVICE, codes
    for call in (lambda: bp.replan(max_iters=1), lambda: bp.expand(1),
                 lambda: bp.solutions(0), lambda: bp.extract_path(0)):
        with pytest.raises(pakr.PakrError) as ei:
            call()
        assert ei.value.code == E_DEVICE
    bp.close()


def test_default_timeout_restored_plans_normally():
    prob = W.config_c2(B=512, A=8, n_cap=20000)
    plan = pakr.Plan(prob)
    plan.replan(max_iters=5)
    assert plan.status()["total_iters"] == 5
    plan.close()
