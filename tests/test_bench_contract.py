"""bench.py's host-side contract (no GPU): the multi-GPU refusal and the
algorithmic FLOP accounting used for the roofline figures."""
import os
import subprocess
import sys

import pytest

from paper_2607_03987_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


@pytest.mark.parametrize("name,table", [(n, W.CONFIGS) for n in ("c1", "c2", "c3", "c4")] +
                         [(n, W.MORE_CONFIGS) for n in W.MORE_CONFIGS])
def test_flop_accounting_covers_every_workload(name, table):
    prob = table[name]()
    f = bench.flops_per_expansion(prob)
    # at least the RK4 state updates of every step (the double integrators'
    # closed-form step: three FMAs per axis)
    per_step = 6 * prob.npos if prob.system in (W.DI2, W.DI3) else 12 * prob.d
    assert f >= prob.T * per_step
    assert bench.nn_flops_per_pair(prob) == 3 * prob.d


def test_flop_accounting_counts_obstacles_and_dynamics():
    base = W.config_c2()
    fewer = base.replace(box_c=base.box_c[:10], box_h=base.box_h[:10])
    assert bench.flops_per_expansion(base) - bench.flops_per_expansion(fewer) == \
        base.T * base.npos * 20
    assert bench.flops_per_expansion(W.config_c4()) > bench.flops_per_expansion(
        W.config_c4().replace(sph_c=W.config_c4().sph_c[:0], sph_r=W.config_c4().sph_r[:0]))
