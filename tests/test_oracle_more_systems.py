"""Pins for the oracle's Dubins airplane and unicycle dynamics (Sec. V-B, V-C).

The paper names the states and controls only; the models are the usual
kinematic ones.  They are pinned by their exact solutions: straight lines
(polynomial in time, where RK4 is exact), constant-rate turns (circles and
helices, approached with observed order 4), and scipy's DOP853 as an
independent integrator under arbitrary held controls.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_2607_03987_amd import workloads as W


def cp_of(name):
    return oracle.CProblem(W.MORE_CONFIGS[name]())


def test_unicycle1_straight_line_exact():
    cp = cp_of("uni1")
    x0 = np.array([2.0, 3.0, 0.4])
    traj = oracle.rollout(cp, x0, np.array([0.35, 0.0]), 20, 0.1)
    for t in range(21):
        s = 0.35 * 0.1 * t
        np.testing.assert_allclose(traj[t], [2 + s * math.cos(0.4), 3 + s * math.sin(0.4), 0.4],
                                   rtol=1e-13, atol=1e-13)


def _uni1_circle_error(h, T_total=2.0):
    cp = cp_of("uni1")
    v, w, th0 = 0.4, 0.3, 0.2
    n = int(round(T_total / h))
    traj = oracle.rollout(cp, np.array([1.0, 2.0, th0]), np.array([v, w]), n, h)
    t = n * h
    exact = [1.0 + v / w * (math.sin(th0 + w * t) - math.sin(th0)),
             2.0 - v / w * (math.cos(th0 + w * t) - math.cos(th0)), th0 + w * t]
    return np.abs(traj[-1] - exact).max()


def test_unicycle1_circle_fourth_order():
    e1, e2 = _uni1_circle_error(0.2), _uni1_circle_error(0.1)
    assert e1 < 1e-6
    assert 12.0 < e1 / e2 < 20.0  # 2^4 = 16 for a fourth-order method


def test_unicycle2_constant_acceleration_exact():
    cp = cp_of("uni2")
    x0 = np.array([1.0, 1.0, 0.7, 0.1, 0.0])
    traj = oracle.rollout(cp, x0, np.array([0.2, 0.0]), 10, 0.1)
    for t in range(11):
        tt = 0.1 * t
        s = 0.1 * tt + 0.5 * 0.2 * tt * tt
        np.testing.assert_allclose(traj[t], [1 + s * math.cos(0.7), 1 + s * math.sin(0.7), 0.7,
                                             0.1 + 0.2 * tt, 0.0], rtol=1e-13, atol=1e-13)


def test_unicycle2_reduces_to_unicycle1_with_zero_controls():
    c1, c2 = cp_of("uni1"), cp_of("uni2")
    a = oracle.rollout(c1, np.array([3.0, 4.0, -0.5]), np.array([0.3, 0.2]), 15, 0.1)
    b = oracle.rollout(c2, np.array([3.0, 4.0, -0.5, 0.3, 0.2]), np.zeros(2), 15, 0.1)
    np.testing.assert_allclose(b[:, :3], a, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(b[:, 3:], np.tile([0.3, 0.2], (16, 1)), rtol=0, atol=0)


def test_dubins_straight_line_exact():
    cp = cp_of("dubins")
    x0 = np.array([1.0, 2.0, 3.0, 0.6, 0.25, 1.5])
    traj = oracle.rollout(cp, x0, np.zeros(3), 20, 0.05)
    d = np.array([math.cos(0.6) * math.cos(0.25), math.sin(0.6) * math.cos(0.25), math.sin(0.25)])
    for t in range(21):
        np.testing.assert_allclose(traj[t, :3], x0[:3] + 1.5 * 0.05 * t * d, rtol=1e-13,
                                   atol=1e-13)
        np.testing.assert_allclose(traj[t, 3:], x0[3:], rtol=0, atol=0)


def _dubins_helix_error(h, T_total=2.0):
    cp = cp_of("dubins")
    v, th, w, ps0 = 1.2, 0.3, 0.5, 0.1
    n = int(round(T_total / h))
    traj = oracle.rollout(cp, np.array([5.0, 5.0, 2.0, ps0, th, v]), np.array([w, 0.0, 0.0]), n, h)
    t = n * h
    rho = v * math.cos(th) / w
    exact = [5.0 + rho * (math.sin(ps0 + w * t) - math.sin(ps0)),
             5.0 - rho * (math.cos(ps0 + w * t) - math.cos(ps0)),
             2.0 + v * math.sin(th) * t, ps0 + w * t, th, v]
    return np.abs(traj[-1] - exact).max()


def test_dubins_helix_fourth_order():
    e1, e2 = _dubins_helix_error(0.2), _dubins_helix_error(0.1)
    assert e1 < 1e-5
    assert 12.0 < e1 / e2 < 20.0


@pytest.mark.parametrize("name,u", [("uni1", [0.45, -0.35]), ("uni2", [0.2, -0.15]),
                                    ("dubins", [0.8, -0.3, 0.4])])
def test_matches_dop853(name, u):
    cp = cp_of(name)
    prob = cp.prob
    x0 = np.asarray(prob.x_init, np.float64).copy()
    if name == "uni2":
        x0[3:] = [0.3, 0.1]
    u = np.asarray(u, np.float64)
    h, n = 0.01, 200

    def rhs(_, x):
        return oracle.dynamics(cp, x, u)

    ref = solve_ivp(rhs, (0.0, h * n), x0, method="DOP853", rtol=1e-12, atol=1e-12).y[:, -1]
    got = oracle.rollout(cp, x0, u, n, h)[-1]
    np.testing.assert_allclose(got, ref, rtol=1e-8, atol=1e-8)


ALL = [("c1", W.CONFIGS), ("c2", W.CONFIGS), ("c3", W.CONFIGS), ("c4", W.CONFIGS),
       ("dubins", W.MORE_CONFIGS), ("uni1", W.MORE_CONFIGS), ("uni2", W.MORE_CONFIGS)]


def _controls(prob, M, rng, spread):
    lo = np.asarray(prob.u_lo, np.float64)[:prob.m]
    hi = np.asarray(prob.u_hi, np.float64)[:prob.m]
    return 0.5 * (lo + hi) + spread * 0.5 * (hi - lo) * rng.uniform(-1, 1, (M, prob.m))


@pytest.mark.parametrize("name,table", ALL)
def test_refinement_dynamics_equal_the_rollout(name, table):
    """The objective's complex-arithmetic copy of f equals f: with only the goal
    term, J is the squared goal distance of the rollout's final position."""
    prob = table[name]().replace(T=6)
    cp = oracle.CProblem(prob)
    rs = W.refine_settings(prob, w_u=0.0, w_c=0.0, w_g=1.0)
    rp = oracle.refine_params(rs.w_u, rs.w_g, rs.w_c, rs.beta, rs.delta, rs.u_ref, rs.u_scale)
    rng = np.random.default_rng(31)
    x = np.asarray(prob.x_init, np.float64)
    U = _controls(prob, 3, rng, 0.3 if name == "c4" else 0.8)
    xs = x
    for e in range(3):
        xs = oracle.rollout(cp, xs, U[e], prob.T, float(prob.dt))[-1]
    want = float(((xs[:prob.npos] - np.asarray(prob.goal_c, np.float64)) ** 2).sum())
    assert oracle.traj_cost(cp, rp, x, U) == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("name", ["dubins", "uni1", "uni2"])
def test_refinement_gradient_matches_finite_differences(name):
    prob = W.MORE_CONFIGS[name]().replace(T=5)
    cp = oracle.CProblem(prob)
    rs = W.refine_settings(prob)
    rp = oracle.refine_params(rs.w_u, rs.w_g, rs.w_c, rs.beta, rs.delta, rs.u_ref, rs.u_scale)
    rng = np.random.default_rng(17)
    x0 = np.asarray(prob.x_init, np.float64)
    U = _controls(prob, 4, rng, 1.0)
    g = oracle.traj_grad(cp, rp, x0, U)
    h = 1e-3 * float(np.mean(rs.u_scale))
    fd = np.zeros_like(U)
    for idx in np.ndindex(*U.shape):
        def d(step):
            Up, Um = U.copy(), U.copy()
            Up[idx] += step
            Um[idx] -= step
            return (oracle.traj_cost(cp, rp, x0, Up) - oracle.traj_cost(cp, rp, x0, Um)) / (2 * step)
        fd[idx] = (4 * d(h / 2) - d(h)) / 3
    assert np.abs(g - fd).max() / max(np.abs(fd).max(), 1e-12) < 1e-6
