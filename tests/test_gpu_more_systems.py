"""The Dubins airplane, the two unicycles, the acrobot and the cart-pole
(Sec. V-A, V-C, V-E) on the GPU.

The same bars as the four main systems: step parity of the planner against the
FP64 reference (several NN tiles and rollout workgroups, a ragged batch), the
refinement's rollout and adjoint against the oracle's objective and
complex-step gradient, a path the planner extracts checked edge by edge by the
oracle, and batched planning of a mix that holds all nine systems, bit-equal
to planning each query alone.
"""
import numpy as np
import pytest

import oracle
from paper_2607_03987_amd import pakr, refine, workloads as W
from tests.parity import CKPT_TOL, GRAD_TOL, rel_err, step_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("name,kw,iters", [
    ("dubins", dict(B=1024, A=8, n_cap=40000), 12),
    ("dubins", dict(B=300, A=3, n_cap=8000, seed=2), 10),
    ("uni1", dict(B=1024, A=8, n_cap=40000), 15),
    ("uni1", dict(B=300, A=3, n_cap=8000, seed=2), 12),
    ("uni2", dict(B=1024, A=8, n_cap=40000), 15),
    ("uni2", dict(B=300, A=3, n_cap=8000, seed=2), 12),
    ("acrobot", dict(B=1024, A=8, n_cap=40000), 15),
    ("acrobot", dict(B=300, A=3, n_cap=8000, seed=2), 12),
    ("cartpole", dict(B=1024, A=8, n_cap=40000), 15),
    ("cartpole", dict(B=300, A=3, n_cap=8000, seed=2), 12),
])
def test_step_parity(name, kw, iters):
    prob = W.MORE_CONFIGS[name](**kw)
    print(f"case {name} {kw}", flush=True)
    stats = step_parity(prob, iters, log=_log)
    assert sum(s["valid"] for s in stats) > 0


@pytest.mark.parametrize("lanes", [1, 4, 16])
@pytest.mark.parametrize("name", ["dubins", "uni2"])
def test_step_parity_lanes(name, lanes):
    prob = W.MORE_CONFIGS[name](B=512, A=8, n_cap=20000)
    print(f"case {name} lanes {lanes}", flush=True)
    step_parity(prob, 6, lanes=lanes, log=_log)


def _controls(prob, n, M, rng, spread):
    lo = np.asarray(prob.u_lo, np.float64)[:prob.m]
    hi = np.asarray(prob.u_hi, np.float64)[:prob.m]
    mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
    return (mid + spread * half * rng.uniform(-1, 1, (n, M, prob.m))).astype(np.float32)


@pytest.mark.parametrize("name,T,M", [("dubins", 20, 5), ("uni1", 10, 6), ("uni2", 10, 6),
                                      ("acrobot", 10, 6), ("cartpole", 10, 6)])
def test_forward_and_adjoint_match_oracle(name, T, M):
    prob = W.MORE_CONFIGS[name]().replace(T=T)
    print(f"case refine {name} T {T} M {M}", flush=True)
    rs = W.refine_settings(prob)
    rp = oracle.refine_params(rs.w_u, rs.w_g, rs.w_c, rs.beta, rs.delta, rs.u_ref, rs.u_scale)
    cp = oracle.CProblem(prob)
    ref = refine.Refiner(prob, rs)
    rng = np.random.default_rng(11)
    n = 6
    U = _controls(prob, n, M, rng, 1.0)
    x0 = np.repeat(np.asarray(prob.x_init, np.float32)[None, :], n, 0)
    x0[:, :prob.npos] += rng.uniform(-0.3, 0.3, (n, prob.npos)).astype(np.float32)
    if name == "uni2":
        x0[:, 3:] = rng.uniform(-0.3, 0.3, (n, 2)).astype(np.float32)
    if name in ("acrobot", "cartpole"):
        x0[:, 2:] = rng.uniform(-1.0, 1.0, (n, 2)).astype(np.float32)
    Ud, x0d = torch.from_numpy(U).cuda(), torch.from_numpy(x0).cuda()
    J, ckpt = ref.forward(x0d, Ud)
    gU = ref.backward(Ud, ckpt, torch.ones(n, device="cuda"))
    J, ckpt, gU = J.cpu().numpy(), ckpt.cpu().numpy(), gU.cpu().numpy()
    for p in range(n):
        x = x0[p].astype(np.float64)
        Jo = oracle.traj_cost(cp, rp, x, U[p].astype(np.float64))
        assert abs(J[p] - Jo) <= 2e-4 * max(abs(Jo), 1.0), (p, J[p], Jo)
        states = [x]
        for e in range(M):
            traj = oracle.rollout(cp, states[-1], U[p, e].astype(np.float64), T, float(prob.dt))
            states.extend(traj[1:])
        ck_err = rel_err(ckpt[p], np.array(states)).max()
        print(f"  traj {p}: checkpoint states max rel err {ck_err:.2e}", flush=True)
        assert ck_err <= CKPT_TOL, (p, ck_err)
        go = oracle.traj_grad(cp, rp, x, U[p].astype(np.float64))
        err = np.linalg.norm(gU[p] - go) / max(np.linalg.norm(go), 1e-12)
        cos = float((gU[p] * go).sum() / (np.linalg.norm(gU[p]) * np.linalg.norm(go) + 1e-30))
        print(f"  traj {p}: J {J[p]:.6g} oracle {Jo:.6g}; grad rel L2 {err:.2e} cos {cos:.8f}",
              flush=True)
        assert err <= GRAD_TOL and cos >= 0.99999, (p, err, cos)
    ref.close()


@pytest.mark.parametrize("name", ["dubins", "uni1", "uni2", "acrobot", "cartpole"])
def test_extracted_path_is_feasible(name):
    prob = W.MORE_CONFIGS[name](max_iters_per_round=400)
    print(f"case path {name}", flush=True)
    plan = pakr.Plan(prob)
    plan.replan(max_rounds=1)
    path = plan.extract_path()
    assert path is not None, plan.status()
    states, actions, cost = path
    assert np.array_equal(states[0], prob.x_init)
    cp = oracle.CProblem(prob)
    total = 0.0
    for e in range(actions.shape[0]):
        ok, xT, c, amb = oracle.edge(cp, states[e].astype(float), total, actions[e].astype(float))
        assert ok or amb, e
        assert rel_err(xT, states[e + 1]).max() <= 1e-4, e
        total = c
    end = states[-1][:prob.npos].astype(np.float64)
    assert np.linalg.norm(end - prob.goal_c) <= prob.goal_r * (1 + 1e-6)
    assert abs(total - cost) <= 1e-4 * max(1.0, cost)
    plan.close()


def test_batch_of_all_nine_systems_equals_single_plans():
    probs = [W.config_c1(seed=1, B=512, A=8), W.config_c2(seed=1, B=512, A=8),
             W.config_c3(seed=1, B=512, A=16), W.config_c4(seed=1, B=256, A=16),
             W.config_dubins(seed=1, B=512, A=8), W.config_uni1(seed=1, B=512, A=8),
             W.config_uni2(seed=1, B=512, A=8), W.config_uni1(seed=2, B=256, A=4),
             W.config_acrobot(seed=1, B=512, A=8), W.config_cartpole(seed=1, B=256, A=4)]
    probs = [p.replace(max_iters_per_round=30, n_cap=min(p.n_cap, 30000), qid=q)
             for q, p in enumerate(probs)]
    print("case batch of the nine systems, teams auto, 2 rounds", flush=True)
    bp = pakr.BatchPlan(probs, lanes=1, teams=0)
    bp.replan(max_rounds=2)
    for q, prob in enumerate(probs):
        pl = pakr.Plan(prob, lanes=1)
        pl.replan(max_rounds=2)
        sb, sp = bp.status(q), pl.status()
        for key in ("total_iters", "expansions", "insertions", "n_nodes", "round", "iter",
                    "n_solutions", "nn_pairs"):
            assert sb[key] == sp[key], (q, prob.name, key, sb[key], sp[key])
        assert [(s["iter"], s["node"], s["cost"]) for s in bp.solutions(q)] == \
               [(s["iter"], s["node"], s["cost"]) for s in pl.solutions()]
        pl.close()
    bp.close()
