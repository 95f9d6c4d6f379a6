"""Pins for the oracle's Dubins airplane, unicycle, acrobot and cart-pole
dynamics (Sec. V-A, V-C, V-E).

The paper names the states and controls only; the models are the usual
kinematic ones for the airplane and the unicycles and the rigid-body ones for
the acrobot and the cart-pole.  They are pinned by exact solutions: straight
lines (polynomial in time, where RK4 is exact), constant-rate turns (circles
and helices, approached with observed order 4), a pole leaning at the angle of
the effective gravity, the nonlinear pendulum's Jacobi-elliptic solution; by
the acrobot's Euler-Lagrange equations taken numerically from its kinematics
and energy (no closed form retyped); by energy conservation; and by scipy's
DOP853 as an independent integrator under arbitrary held controls.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.special import ellipj, ellipk

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


def _acrobot_energy(dyn, x):
    """Kinetic plus potential energy from the link kinematics (height up)."""
    m1, m2, l1, lc1, lc2, I1, I2, g = dyn
    q1, q2, w1, w2 = x
    # centres of mass; angles from the downward vertical, the second relative
    p1 = np.array([lc1 * math.sin(q1), -lc1 * math.cos(q1)])
    v1 = np.array([lc1 * math.cos(q1), lc1 * math.sin(q1)]) * w1
    p2 = np.array([l1 * math.sin(q1) + lc2 * math.sin(q1 + q2),
                   -l1 * math.cos(q1) - lc2 * math.cos(q1 + q2)])
    v2 = (np.array([l1 * math.cos(q1), l1 * math.sin(q1)]) * w1
          + np.array([lc2 * math.cos(q1 + q2), lc2 * math.sin(q1 + q2)]) * (w1 + w2))
    T = 0.5 * m1 * v1 @ v1 + 0.5 * I1 * w1 ** 2 + 0.5 * m2 * v2 @ v2 + 0.5 * I2 * (w1 + w2) ** 2
    return T, m1 * g * p1[1] + m2 * g * p2[1]


def _acrobot_euler_lagrange(dyn, x, tau):
    """q'' from d/dt dL/dq' - dL/dq = (0, tau), with every derivative of
    L = T - V taken by central differences of the energy function."""
    def L(q, w):
        T, V = _acrobot_energy(dyn, np.concatenate([q, w]))
        return T - V
    q, w = np.asarray(x[:2], float), np.asarray(x[2:], float)
    # steps: L is quadratic in q', so differences in q' are exact for any step
    # (a large one keeps rounding small); differences in q are O(hq^2)
    hw, hq = 0.1, 1e-4
    E = np.eye(2)
    M = np.array([[(L(q, w + hw * (E[i] + E[j])) - L(q, w + hw * (E[i] - E[j]))
                    - L(q, w - hw * (E[i] - E[j])) + L(q, w - hw * (E[i] + E[j]))) / (4 * hw * hw)
                   for j in range(2)] for i in range(2)])
    dLdq = np.array([(L(q + hq * E[i], w) - L(q - hq * E[i], w)) / (2 * hq) for i in range(2)])
    # d/dt dL/dq' = M q'' + (d2L/dq' dq) q'
    C = np.array([[(L(q + hq * E[j], w + hw * E[i]) - L(q + hq * E[j], w - hw * E[i])
                    - L(q - hq * E[j], w + hw * E[i]) + L(q - hq * E[j], w - hw * E[i]))
                   / (4 * hq * hw) for j in range(2)] for i in range(2)])
    return np.linalg.solve(M, np.array([0.0, tau]) + dLdq - C @ w)


@pytest.mark.parametrize("x,tau", [([0.3, -0.7, 1.1, -2.0], 0.0), ([2.5, 1.2, -3.0, 0.4], 4.0),
                                   ([-1.0, 2.9, 0.0, 5.5], -7.5), ([0.0, 0.0, 0.0, 0.0], 10.0)])
def test_acrobot_matches_euler_lagrange_of_its_kinematics(x, tau):
    cp = cp_of("acrobot")
    dyn = np.asarray(cp.prob.dyn, np.float64)
    got = oracle.dynamics(cp, np.array(x), np.array([tau]))
    np.testing.assert_allclose(got[:2], x[2:], rtol=0, atol=0)
    np.testing.assert_allclose(got[2:], _acrobot_euler_lagrange(dyn, x, tau), rtol=1e-7, atol=1e-7)


def test_acrobot_conserves_energy_without_torque():
    cp = cp_of("acrobot")
    dyn = np.asarray(cp.prob.dyn, np.float64)
    x0 = np.array([2.0, -1.0, 0.5, 1.5])
    traj = oracle.rollout(cp, x0, np.zeros(1), 2000, 1e-3)
    E = [sum(_acrobot_energy(dyn, x)) for x in traj[::100]]
    assert np.ptp(E) < 1e-8 * max(1.0, abs(E[0]))
    assert np.abs(traj[-1] - x0).max() > 0.5  # it did move


def test_cartpole_leans_at_the_effective_gravity_angle():
    """Constant acceleration a: the pole at atan(a/g) from upright, at rest,
    stays there while the cart moves as x0 + v0 t + a t^2 / 2 (exact for RK4)."""
    cp = cp_of("cartpole")
    a, g = 3.0, float(cp.prob.dyn[1])
    th = math.atan2(a, g)
    x0 = np.array([0.5, th, -0.2, 0.0])
    traj = oracle.rollout(cp, x0, np.array([a]), 50, 0.02)
    for t in range(51):
        tt = 0.02 * t
        np.testing.assert_allclose(traj[t], [0.5 - 0.2 * tt + 0.5 * a * tt * tt, th, -0.2 + a * tt, 0.0],
                                   rtol=1e-12, atol=1e-12)


def test_cartpole_hanging_pole_is_the_nonlinear_pendulum():
    """a = 0, released at rest phi0 from hanging: phi(t) = 2 asin(k sn(K - w t, k^2)),
    k = sin(phi0 / 2), w = sqrt(g / l) (Jacobi elliptic solution)."""
    cp = cp_of("cartpole")
    l, g = float(cp.prob.dyn[0]), float(cp.prob.dyn[1])
    phi0 = 1.2
    x0 = np.array([0.0, math.pi + phi0, 0.0, 0.0])
    h, n = 1e-3, 3000
    traj = oracle.rollout(cp, x0, np.zeros(1), n, h)
    k = math.sin(phi0 / 2)
    K = ellipk(k * k)
    w = math.sqrt(g / l)
    for t in range(0, n + 1, 250):
        sn = ellipj(K - w * h * t, k * k)[0]
        assert traj[t, 1] - math.pi == pytest.approx(2 * math.asin(k * sn), abs=1e-9)
    E = 0.5 * l * l * traj[:, 3] ** 2 + g * l * np.cos(traj[:, 1])
    assert np.ptp(E) < 1e-9


@pytest.mark.parametrize("name,u", [("uni1", [0.45, -0.35]), ("uni2", [0.2, -0.15]),
                                    ("dubins", [0.8, -0.3, 0.4]), ("acrobot", [3.0]),
                                    ("cartpole", [-4.0])])
def test_matches_dop853(name, u):
    cp = cp_of(name)
    prob = cp.prob
    x0 = np.asarray(prob.x_init, np.float64).copy()
    if name == "uni2":
        x0[3:] = [0.3, 0.1]
    if name in ("acrobot", "cartpole"):
        x0[2:] = [0.7, -1.3]
    u = np.asarray(u, np.float64)
    # the pendulum systems accelerate faster: a smaller step keeps RK4's error
    # below the tolerance over the same 2 s
    h, n = (0.001, 2000) if name in ("acrobot", "cartpole") else (0.01, 200)

    def rhs(_, x):
        return oracle.dynamics(cp, x, u)

    ref = solve_ivp(rhs, (0.0, h * n), x0, method="DOP853", rtol=1e-12, atol=1e-12).y[:, -1]
    got = oracle.rollout(cp, x0, u, n, h)[-1]
    np.testing.assert_allclose(got, ref, rtol=1e-8, atol=1e-8)


ALL = [("c1", W.CONFIGS), ("c2", W.CONFIGS), ("c3", W.CONFIGS), ("c4", W.CONFIGS),
       ("dubins", W.MORE_CONFIGS), ("uni1", W.MORE_CONFIGS), ("uni2", W.MORE_CONFIGS),
       ("acrobot", W.MORE_CONFIGS), ("cartpole", W.MORE_CONFIGS)]


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


@pytest.mark.parametrize("name", ["dubins", "uni1", "uni2", "acrobot", "cartpole"])
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
