"""Pins for the oracle's trajectory-refinement objective and its gradient.

The objective (effort + terminal goal term + softplus obstacle/bound
penalty summed over the sub-step states of a piecewise-constant control
sequence rolled out with RK4) and its FP64 gradient, obtained by complex-step
differentiation, are pinned against:
  - the closed form of J and dJ/dU for the double integrator without the
    penalty (RK4 is exact for piecewise-constant acceleration);
  - signed distances fixed by geometry (points at known distances from a
    sphere, a box face, a box corner, a wall; known speeds and limits);
  - Richardson-extrapolated central finite differences on every system;
  - torch.autograd.gradcheck on the FP64 oracle wrapped as a Function.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2607_03987_amd import workloads as W


def sp(z, beta):
    """softplus_beta(z) = log(1 + exp(beta z)) / beta, by definition."""
    return math.log1p(math.exp(beta * z)) / beta if beta * z < 30 else z + math.log1p(
        math.exp(-beta * z)) / beta


def rp_of(rs):
    return oracle.refine_params(rs.w_u, rs.w_g, rs.w_c, rs.beta, rs.delta, rs.u_ref, rs.u_scale)


def controls(prob, M, rng, spread=1.0):
    lo = np.asarray(prob.u_lo, np.float64)[:prob.m]
    hi = np.asarray(prob.u_hi, np.float64)[:prob.m]
    mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
    return mid + spread * half * rng.uniform(-1, 1, (M, prob.m))


# --- closed form: double integrator without the penalty ----------------------

@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_double_integrator_closed_form(cfg):
    prob = W.CONFIGS[cfg]().replace(T=7)
    cp = oracle.CProblem(prob)
    D = prob.npos
    rs = W.refine_settings(prob, w_c=0.0, w_u=0.7, w_g=3.0, u_ref=(0.1,) * D,
                           u_scale=(0.5,) * D)
    rp = rp_of(rs)
    rng = np.random.default_rng(3)
    for M in (1, 4):
        x0 = np.concatenate([rng.uniform(2, 8, D), rng.uniform(-1, 1, D)])
        U = rng.uniform(-1, 1, (M, D))
        tau = prob.T * float(prob.dt)       # edge duration
        T_end = M * tau
        w = np.array([tau * (T_end - (e + 1) * tau) + 0.5 * tau * tau for e in range(M)])
        pN = x0[:D] + x0[D:] * T_end + (w[:, None] * U).sum(0)
        r = pN - np.asarray(prob.goal_c, np.float64)
        J = rs.w_u * tau * (((U - 0.1) / 0.5) ** 2).sum() + rs.w_g * (r ** 2).sum()
        grad = 2 * rs.w_u * tau * (U - 0.1) / 0.25 + 2 * rs.w_g * w[:, None] * r[None, :]
        assert oracle.traj_cost(cp, rp, x0, U) == pytest.approx(J, rel=1e-12)
        np.testing.assert_allclose(oracle.traj_grad(cp, rp, x0, U), grad, rtol=1e-10, atol=1e-10)


# --- penalty: signed distances fixed by geometry ------------------------------

def _one_state_penalty(prob, x, beta=20.0, delta=0.1):
    """J of one RK4 step with zero velocity and control: pen(x) alone."""
    prob = prob.replace(T=1)
    cp = oracle.CProblem(prob)
    rs = W.refine_settings(prob, w_u=0.0, w_g=0.0, w_c=1.0, beta=beta, delta=delta)
    U = np.zeros((1, prob.m))
    return oracle.traj_cost(cp, rp_of(rs), np.asarray(x, np.float64), U)


def _di3_scene(box_c=(), box_h=(), sph_c=(), sph_r=(), ws=(0, 100)):
    return W.build_problem(W.DI3, [ws[0]] * 3, [ws[1]] * 3, np.array(box_c).reshape(-1, 3),
                           np.array(box_h).reshape(-1, 3), np.array(sph_c).reshape(-1, 3),
                           np.array(sph_r), [50, 50, 50, 0, 0, 0], [60, 60, 60], 1.0, B=64,
                           A=4, T=1, dt=np.float32(0.05), n_cap=1024,
                           cost_kind=W.COST_DURATION).replace(vnorm_max=np.float32(0))


def _wall_terms(x, lo, hi, beta):
    return sum(sp(x[c] - hi, beta) + sp(lo - x[c], beta) for c in range(3))


@pytest.mark.parametrize("dist", [0.3, 1.2, 2.0, 2.05, 2.2, 3.5])
def test_sphere_signed_distance(dist):
    prob = _di3_scene(sph_c=[[40, 40, 40]], sph_r=[2.0])
    direction = np.array([2.0, -1.0, 2.0]) / 3.0
    x = np.concatenate([np.array([40, 40, 40]) + dist * direction, np.zeros(3)])
    want = sp(0.1 - (dist - 2.0), 20.0) + _wall_terms(x, 0, 100, 20.0)
    assert _one_state_penalty(prob, x) == pytest.approx(want, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("x,sd", [
    ([30.0, 30.0, 30.0], -1.0),          # centre: nearest face is the z face (half 1)
    ([30.0, 30.0, 30.8], -0.2),          # 0.2 below the top face
    ([32.7, 30.0, 30.0], -0.3),          # 0.3 inside the x face (half 3)
    ([33.5, 30.0, 30.0], 0.5),           # 0.5 outside the x face
    ([33.3, 32.4, 31.0], 0.5),           # outside an edge: (0.3, 0.4, 0) -> 0.5
    ([34.0, 34.0, 33.0], 3.0),           # outside a corner: (1, 2, 2) -> 3
])
def test_box_signed_distance(x, sd):
    prob = _di3_scene(box_c=[[30, 30, 30]], box_h=[[3, 2, 1]])
    xs = np.array(x + [0, 0, 0], np.float64)
    want = sp(0.1 - sd, 20.0) + _wall_terms(xs, 0, 100, 20.0)
    assert _one_state_penalty(prob, xs) == pytest.approx(want, rel=1e-12, abs=1e-15)


def test_workspace_wall_terms():
    prob = _di3_scene(ws=(0, 10))
    x = np.array([0.05, 9.9, 5.0, 0, 0, 0])
    want = sp(-0.05, 20) + sp(0.05 - 10, 20) + sp(9.9 - 10, 20) + sp(-9.9, 20) + \
        sp(5 - 10, 20) + sp(-5, 20)
    assert _one_state_penalty(prob, x) == pytest.approx(want, rel=1e-12)
    outside = np.array([-0.5, 5, 5, 0, 0, 0])
    assert _one_state_penalty(prob, outside) > 0.5  # a violation costs about its depth


def test_speed_and_limit_terms():
    # double integrator: |v| = 2.5 against vnorm_max 2; one step of length h
    prob = W.config_c2().replace(box_c=np.zeros((0, 3), np.float32),
                                 box_h=np.zeros((0, 3), np.float32), T=1)
    h = float(prob.dt)
    v = np.array([1.5, 2.0, 0.0])
    x0 = np.concatenate([[5.0, 5.0, 5.0], v])
    x1 = np.concatenate([x0[:3] + v * h, v])
    want = sp(2.5 - 2.0, 20) + _wall_terms(x1, 0, 10, 20)
    assert _one_state_penalty(prob, x0) == pytest.approx(want, rel=1e-12)
    # car: speed 1.3 above v_max 1 and steering 0.7 above 0.6 (held: zero controls)
    car = W.config_c3().replace(box_c=np.zeros((0, 2), np.float32),
                                box_h=np.zeros((0, 2), np.float32), T=1)
    lo, hi = np.asarray(car.lim_lo, np.float64), np.asarray(car.lim_hi, np.float64)
    x = np.array([5.0, 5.0, 0.0, 1.3, 0.7])
    cp = oracle.CProblem(car)
    x1 = oracle.rollout(cp, x, np.zeros(2), 1, float(car.dt))[-1]
    want = sum(sp(x1[i] - hi[i], 20) + sp(lo[i] - x1[i], 20) for i in range(2, 5)
               if np.isfinite(hi[i])) + sum(sp(x1[c] - float(car.ws_hi[c]), 20) +
                                            sp(float(car.ws_lo[c]) - x1[c], 20) for c in range(2))
    assert _one_state_penalty(car, x) == pytest.approx(want, rel=1e-12)


# --- gradient: finite differences and gradcheck --------------------------------

def _fd_richardson(f, U, h):
    g = np.zeros_like(U)
    for idx in np.ndindex(*U.shape):
        def d(step):
            Up, Um = U.copy(), U.copy()
            Up[idx] += step
            Um[idx] -= step
            return (f(Up) - f(Um)) / (2 * step)
        g[idx] = (4 * d(h / 2) - d(h)) / 3
    return g


@pytest.mark.parametrize("cfg,T,spread", [("c1", 5, 1.0), ("c2", 5, 1.0), ("c3", 6, 1.0),
                                          ("c4", 8, 0.3)])
def test_gradient_matches_finite_differences(cfg, T, spread):
    prob = W.CONFIGS[cfg]().replace(T=T)
    cp = oracle.CProblem(prob)
    rs = W.refine_settings(prob)
    rp = rp_of(rs)
    rng = np.random.default_rng(11)
    x0 = np.asarray(prob.x_init, np.float64)
    for trial in range(2):
        U = controls(prob, 4, rng, spread)
        g = oracle.traj_grad(cp, rp, x0, U)
        scale = np.asarray(rs.u_scale)[None, :]
        fd = _fd_richardson(lambda V: oracle.traj_cost(cp, rp, x0, V), U, 1e-3 * scale.mean())
        err = np.abs(g - fd).max() / max(np.abs(fd).max(), 1e-12)
        assert err < 1e-6, (cfg, trial, err)


def test_gradcheck_on_fp64_oracle():
    prob = W.config_c4().replace(T=3)
    cp = oracle.CProblem(prob)
    rp = rp_of(W.refine_settings(prob))
    x0 = np.asarray(prob.x_init, np.float64)

    class OracleJ(torch.autograd.Function):
        @staticmethod
        def forward(ctx, U):
            ctx.save_for_backward(U)
            return torch.tensor(oracle.traj_cost(cp, rp, x0, U.detach().numpy()),
                                dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            (U,) = ctx.saved_tensors
            return gJ * torch.from_numpy(oracle.traj_grad(cp, rp, x0, U.detach().numpy()))

    rng = np.random.default_rng(5)
    U = torch.tensor(controls(prob, 3, rng, 0.3), dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(OracleJ.apply, (U,), eps=1e-6, atol=1e-6, rtol=1e-5)


def test_descent_direction_lowers_cost():
    prob = W.config_c3().replace(T=10)
    cp = oracle.CProblem(prob)
    rp = rp_of(W.refine_settings(prob))
    x0 = np.asarray(prob.x_init, np.float64)
    U = controls(prob, 5, np.random.default_rng(2))
    g = oracle.traj_grad(cp, rp, x0, U)
    J0 = oracle.traj_cost(cp, rp, x0, U)
    J1 = oracle.traj_cost(cp, rp, x0, U - 1e-4 * g / np.linalg.norm(g))
    assert J1 < J0
