"""Synthetic planning problems: system tables, scene generation, workload configs.

This module holds input data only.  It contains none of the planner's
arithmetic (no dynamics, no sampling streams, no collision tests); both the
HIP path and the FP64 reference consume the ``Problem`` objects built here.

The paper evaluates on environments and benchmark problems that are not
reproduced here (Sec. V-A, V-C); the scenes below are seeded random stand-ins
with the same shape: a bounded 2D/3D workspace cluttered with axis-aligned
boxes, discs or spheres, a start state and a spherical goal region
(problem statement, Sec. III).

All real-valued fields are float32: the planner is defined on these exact
values, and the reference reads them as exact doubles.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# System identifiers shared by the C ABI (include/pakr.h) and the reference.
DI2, DI3, CAR, QUAD, DUBINS, UNI1, UNI2, ACROBOT, CARTPOLE = 0, 1, 2, 3, 4, 5, 6, 7, 8
SYSTEM_NAMES = {DI2: "di2", DI3: "di3", CAR: "car", QUAD: "quad", DUBINS: "dubins",
                UNI1: "uni1", UNI2: "uni2", ACROBOT: "acrobot", CARTPOLE: "cartpole"}

# Cost kinds (problem statement, Sec. III: path length or time optimality).
COST_DURATION, COST_PATH_LENGTH = 0, 1
# Heuristic kinds for the cost-bounded prune of Alg. 1.
H_ADMISSIBLE, H_PAPER_LITERAL, H_NONE = 0, 1, 2

F32_INF = np.float32(np.inf)


@dataclasses.dataclass
class Problem:
    """One planning query: dynamics, scene, start, goal and planner settings."""

    system: int
    d: int
    m: int
    npos: int
    dyn: np.ndarray            # float32[8]   dynamics constants (see system_table)
    sample_lo: np.ndarray      # float32[d]   SampleStates box
    sample_hi: np.ndarray
    u_lo: np.ndarray           # float32[m]   control box U
    u_hi: np.ndarray
    lim_lo: np.ndarray         # float32[d]   per-dimension state limits (+-inf: none)
    lim_hi: np.ndarray
    vnorm_max: np.float32      # speed-norm limit on the velocity block (0: none)
    ws_lo: np.ndarray          # float32[npos] workspace box (closed)
    ws_hi: np.ndarray
    box_c: np.ndarray          # float32[nb, npos] axis-aligned boxes: centre
    box_h: np.ndarray          # float32[nb, npos]                      half extent
    sph_c: np.ndarray          # float32[ns, npos] spheres (discs in 2D): centre
    sph_r: np.ndarray          # float32[ns]                             radius
    goal_c: np.ndarray         # float32[npos]
    goal_r: np.float32
    x_init: np.ndarray         # float32[d]
    B: int = 256               # rollouts per iteration
    A: int = 4                 # branching factor (controls per selected parent)
    T: int = 10                # RK4 steps per edge, control held
    dt: np.float32 = np.float32(0.05)
    n_cap: int = 16384
    cost_kind: int = COST_PATH_LENGTH
    h_kind: int = H_ADMISSIBLE
    h_speed: np.float32 = np.float32(1.0)   # divisor that makes h admissible for duration cost
    c0: float = math.inf                    # initial cost bound
    seed: int = 0
    qid: int = 0
    max_iters_per_round: int = 100000
    name: str = ""

    @property
    def K(self) -> int:
        return self.B // self.A

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def _f32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float32)


def system_table(system: int, ws_lo, ws_hi) -> dict:
    """Per-system constants: state/control sizes, sampling box, limits, dynamics."""
    ws_lo = _f32(ws_lo)
    ws_hi = _f32(ws_hi)
    inf = np.inf
    pi = math.pi
    if system in (DI2, DI3):
        D = 2 if system == DI2 else 3
        d, m = 2 * D, D
        s_lo = np.concatenate([ws_lo, np.full(D, -2.0)])
        s_hi = np.concatenate([ws_hi, np.full(D, 2.0)])
        return dict(d=d, m=m, npos=D, dyn=np.zeros(8),
                    sample_lo=s_lo, sample_hi=s_hi,
                    u_lo=np.full(m, -1.0), u_hi=np.full(m, 1.0),
                    lim_lo=np.full(d, -inf), lim_hi=np.full(d, inf),
                    vnorm_max=2.0, h_speed=2.0)
    if system == CAR:
        # state (x, y, theta, v, phi); control (acceleration, steering rate)
        d, m = 5, 2
        s_lo = [ws_lo[0], ws_lo[1], -pi, -1.0, -0.6]
        s_hi = [ws_hi[0], ws_hi[1], pi, 1.0, 0.6]
        lim_lo = [-inf, -inf, -inf, -1.0, -0.6]
        lim_hi = [inf, inf, inf, 1.0, 0.6]
        dyn = np.zeros(8)
        dyn[0] = 1.0  # wheelbase
        return dict(d=d, m=m, npos=2, dyn=dyn, sample_lo=s_lo, sample_hi=s_hi,
                    u_lo=[-1.0, -0.5], u_hi=[1.0, 0.5], lim_lo=lim_lo, lim_hi=lim_hi,
                    vnorm_max=0.0, h_speed=1.0)
    if system == QUAD:
        # state (x,y,z, roll,pitch,yaw, u,v,w body velocity, p,q,r body rates)
        # control (thrust, tau_x, tau_y, tau_z); m=1, g=9.81, I=diag(.01,.01,.02)
        d, m = 12, 4
        mass, g = 1.0, 9.81
        ang, vel, rate = 1.2, 3.0, 5.0
        s_lo = [ws_lo[0], ws_lo[1], ws_lo[2], -ang, -ang, -pi,
                -vel, -vel, -vel, -rate, -rate, -rate]
        s_hi = [ws_hi[0], ws_hi[1], ws_hi[2], ang, ang, pi,
                vel, vel, vel, rate, rate, rate]
        lim_lo = [-inf, -inf, -inf, -ang, -ang, -inf,
                  -vel, -vel, -vel, -rate, -rate, -rate]
        lim_hi = [inf, inf, inf, ang, ang, inf, vel, vel, vel, rate, rate, rate]
        dyn = np.zeros(8)
        dyn[:5] = [mass, g, 0.01, 0.01, 0.02]
        thrust_max = float(np.float32(2.0 * mass * g))
        return dict(d=d, m=m, npos=3, dyn=dyn, sample_lo=s_lo, sample_hi=s_hi,
                    u_lo=[0.0, -0.1, -0.1, -0.1], u_hi=[thrust_max, 0.1, 0.1, 0.1],
                    lim_lo=lim_lo, lim_hi=lim_hi, vnorm_max=0.0,
                    h_speed=float(np.float32(math.sqrt(3.0) * vel)))
    if system == DUBINS:
        # Dubins airplane: state (x,y,z, yaw, pitch, speed); control (yaw rate,
        # pitch rate, acceleration); pitch within +-0.6, speed in [0.5, 2]
        d, m = 6, 3
        s_lo = [ws_lo[0], ws_lo[1], ws_lo[2], -pi, -0.6, 0.5]
        s_hi = [ws_hi[0], ws_hi[1], ws_hi[2], pi, 0.6, 2.0]
        lim_lo = [-inf, -inf, -inf, -inf, -0.6, 0.5]
        lim_hi = [inf, inf, inf, inf, 0.6, 2.0]
        return dict(d=d, m=m, npos=3, dyn=np.zeros(8), sample_lo=s_lo, sample_hi=s_hi,
                    u_lo=[-1.0, -0.5, -0.5], u_hi=[1.0, 0.5, 0.5], lim_lo=lim_lo,
                    lim_hi=lim_hi, vnorm_max=0.0, h_speed=2.0)
    if system == UNI1:
        # unicycle 1: state (x, y, heading); control (speed, turn rate)
        s_lo = [ws_lo[0], ws_lo[1], -pi]
        s_hi = [ws_hi[0], ws_hi[1], pi]
        return dict(d=3, m=2, npos=2, dyn=np.zeros(8), sample_lo=s_lo, sample_hi=s_hi,
                    u_lo=[-0.5, -0.5], u_hi=[0.5, 0.5], lim_lo=[-inf] * 3, lim_hi=[inf] * 3,
                    vnorm_max=0.0, h_speed=0.5)
    if system == UNI2:
        # unicycle 2: state (x, y, heading, speed, turn rate); control
        # (acceleration, angular acceleration); |speed|, |turn rate| <= 0.5
        s_lo = [ws_lo[0], ws_lo[1], -pi, -0.5, -0.5]
        s_hi = [ws_hi[0], ws_hi[1], pi, 0.5, 0.5]
        return dict(d=5, m=2, npos=2, dyn=np.zeros(8), sample_lo=s_lo, sample_hi=s_hi,
                    u_lo=[-0.25, -0.25], u_hi=[0.25, 0.25],
                    lim_lo=[-inf, -inf, -inf, -0.5, -0.5], lim_hi=[inf, inf, inf, 0.5, 0.5],
                    vnorm_max=0.0, h_speed=0.5)
    if system == ACROBOT:
        # acrobot: configuration (shoulder angle from hanging, elbow angle);
        # uniform links m 1, length 1, centre of mass at 0.5, I = 1/12 about
        # it; |joint rates| <= 8, |elbow torque| <= 10
        rate = 8.0
        s_lo = [ws_lo[0], ws_lo[1], -rate, -rate]
        s_hi = [ws_hi[0], ws_hi[1], rate, rate]
        dyn = np.zeros(8)
        dyn[:8] = [1.0, 1.0, 1.0, 0.5, 0.5, 1.0 / 12.0, 1.0 / 12.0, 9.81]
        return dict(d=4, m=1, npos=2, dyn=dyn, sample_lo=s_lo, sample_hi=s_hi,
                    u_lo=[-10.0], u_hi=[10.0], lim_lo=[-inf, -inf, -rate, -rate],
                    lim_hi=[inf, inf, rate, rate], vnorm_max=0.0,
                    h_speed=float(np.float32(math.sqrt(2.0) * rate)))
    if system == CARTPOLE:
        # cart-pole: configuration (cart position, pole angle from upright);
        # pole length 1, g 9.81; |cart speed| <= 4, |pole rate| <= 10, cart
        # acceleration in [-10, 10]
        vmax, wmax = 4.0, 10.0
        s_lo = [ws_lo[0], ws_lo[1], -vmax, -wmax]
        s_hi = [ws_hi[0], ws_hi[1], vmax, wmax]
        dyn = np.zeros(8)
        dyn[:2] = [1.0, 9.81]
        return dict(d=4, m=1, npos=2, dyn=dyn, sample_lo=s_lo, sample_hi=s_hi,
                    u_lo=[-10.0], u_hi=[10.0], lim_lo=[-inf, -inf, -vmax, -wmax],
                    lim_hi=[inf, inf, vmax, wmax], vnorm_max=0.0,
                    h_speed=float(np.float32(math.hypot(vmax, wmax))))
    raise ValueError(f"unknown system {system}")


def _clear_of(kind: str, c, h_or_r, p, clearance: float) -> bool:
    """True when the obstacle keeps more than `clearance` away from point p."""
    c = np.asarray(c, np.float64)
    p = np.asarray(p, np.float64)
    if kind == "box":
        gap = np.maximum(np.abs(p - c) - np.asarray(h_or_r, np.float64), 0.0)
        return float(np.sqrt(np.sum(gap * gap))) > clearance
    return float(np.sqrt(np.sum((p - c) ** 2))) - float(h_or_r) > clearance


def make_scene(rng: np.random.Generator, ws_lo, ws_hi, n_box: int, box_side, n_sph: int,
               sph_r, start_pos, goal_c, goal_r: float, square: bool = False):
    """Random axis-aligned boxes and spheres, redrawn while too close to start or goal.

    A box (sphere) is redrawn if it comes within 0.5 of the start position or
    within goal_r + 0.5 of the goal centre.  square: boxes with equal sides.
    """
    ws_lo = np.asarray(ws_lo, np.float64)
    ws_hi = np.asarray(ws_hi, np.float64)
    D = ws_lo.size
    boxes_c, boxes_h, sph_cs, sph_rs = [], [], [], []
    for _ in range(n_box):
        while True:
            side = (np.full(D, rng.uniform(box_side[0], box_side[1])) if square
                    else rng.uniform(box_side[0], box_side[1], size=D))
            c = rng.uniform(ws_lo, ws_hi)
            h = 0.5 * side
            if (_clear_of("box", c, h, start_pos, 0.5)
                    and _clear_of("box", c, h, goal_c, goal_r + 0.5)):
                break
        boxes_c.append(c)
        boxes_h.append(h)
    for _ in range(n_sph):
        while True:
            r = rng.uniform(sph_r[0], sph_r[1])
            c = rng.uniform(ws_lo, ws_hi)
            if (_clear_of("sph", c, r, start_pos, 0.5)
                    and _clear_of("sph", c, r, goal_c, goal_r + 0.5)):
                break
        sph_cs.append(c)
        sph_rs.append(r)
    box_c = _f32(boxes_c).reshape(-1, D)
    box_h = _f32(boxes_h).reshape(-1, D)
    sph_c = _f32(sph_cs).reshape(-1, D)
    sph_r = _f32(sph_rs).reshape(-1)
    return box_c, box_h, sph_c, sph_r


def build_problem(system: int, ws_lo, ws_hi, box_c, box_h, sph_c, sph_r, x_init, goal_c,
                  goal_r, **params) -> Problem:
    t = system_table(system, ws_lo, ws_hi)
    return Problem(
        system=system, d=t["d"], m=t["m"], npos=t["npos"], dyn=_f32(t["dyn"]),
        sample_lo=_f32(t["sample_lo"]), sample_hi=_f32(t["sample_hi"]),
        u_lo=_f32(t["u_lo"]), u_hi=_f32(t["u_hi"]),
        lim_lo=_f32(t["lim_lo"]), lim_hi=_f32(t["lim_hi"]),
        vnorm_max=np.float32(t["vnorm_max"]),
        ws_lo=_f32(ws_lo), ws_hi=_f32(ws_hi),
        box_c=_f32(box_c).reshape(-1, t["npos"]), box_h=_f32(box_h).reshape(-1, t["npos"]),
        sph_c=_f32(sph_c).reshape(-1, t["npos"]), sph_r=_f32(sph_r).reshape(-1),
        goal_c=_f32(goal_c), goal_r=np.float32(goal_r), x_init=_f32(x_init),
        h_speed=np.float32(params.pop("h_speed", t["h_speed"])), **params)


# ----------------------------------------------------------------------------
# The five workload configurations (single queries c1-c4, batched c5).
# ----------------------------------------------------------------------------

def config_c1(seed: int = 0, **over) -> Problem:
    """2D double integrator, [0,10]^2, 10 boxes side U(0.5,2); B 256, A 4, T 10, dt .05."""
    rng = np.random.default_rng([seed, 1])
    start = [1.0, 1.0, 0.0, 0.0]
    goal_c, goal_r = [9.0, 9.0], 0.5
    scene = make_scene(rng, [0, 0], [10, 10], 10, (0.5, 2.0), 0, (0, 0), start[:2], goal_c,
                       goal_r)
    kw = dict(B=256, A=4, T=10, dt=np.float32(0.05), n_cap=16384, cost_kind=COST_PATH_LENGTH,
              seed=seed, name="c1_di2")
    kw.update(over)
    return build_problem(DI2, [0, 0], [10, 10], *scene, start, goal_c, goal_r, **kw)


def config_c2(seed: int = 0, **over) -> Problem:
    """3D double integrator, [0,10]^3, 30 boxes side U(0.5,2.5); B 4096, A 8, T 20, dt .05."""
    rng = np.random.default_rng([seed, 2])
    start = [1.0, 1.0, 1.0, 0.0, 0.0, 0.0]
    goal_c, goal_r = [9.0, 9.0, 9.0], 0.5
    scene = make_scene(rng, [0, 0, 0], [10, 10, 10], 30, (0.5, 2.5), 0, (0, 0), start[:3],
                       goal_c, goal_r)
    kw = dict(B=4096, A=8, T=20, dt=np.float32(0.05), n_cap=262144, cost_kind=COST_DURATION,
              seed=seed, name="c2_di3")
    kw.update(over)
    return build_problem(DI3, [0, 0, 0], [10, 10, 10], *scene, start, goal_c, goal_r, **kw)


def config_c3(seed: int = 0, **over) -> Problem:
    """Second-order car, [0,20]^2, 60 boxes + 20 discs; B 8192, A 16, T 25, dt .04."""
    rng = np.random.default_rng([seed, 3])
    start = [1.0, 1.0, 0.0, 0.0, 0.0]
    goal_c, goal_r = [19.0, 19.0], 1.0
    scene = make_scene(rng, [0, 0], [20, 20], 60, (0.5, 2.0), 20, (0.3, 1.0), start[:2],
                       goal_c, goal_r)
    kw = dict(B=8192, A=16, T=25, dt=np.float32(0.04), n_cap=1 << 20, cost_kind=COST_DURATION,
              seed=seed, name="c3_car")
    kw.update(over)
    return build_problem(CAR, [0, 0], [20, 20], *scene, start, goal_c, goal_r, **kw)


def config_c4(seed: int = 0, **over) -> Problem:
    """12D quadrotor, [0,10]^3, 50 spheres r U(0.3,1.2); B 8192, A 16, T 40, dt .02."""
    rng = np.random.default_rng([seed, 4])
    start = [1.0, 1.0, 1.0] + [0.0] * 9
    goal_c, goal_r = [9.0, 9.0, 9.0], 1.0
    scene = make_scene(rng, [0, 0, 0], [10, 10, 10], 0, (0, 0), 50, (0.3, 1.2), start[:3],
                       goal_c, goal_r)
    kw = dict(B=8192, A=16, T=40, dt=np.float32(0.02), n_cap=1 << 20, cost_kind=COST_DURATION,
              seed=seed, name="c4_quad")
    kw.update(over)
    return build_problem(QUAD, [0, 0, 0], [10, 10, 10], *scene, start, goal_c, goal_r, **kw)


CONFIGS = {"c1": config_c1, "c2": config_c2, "c3": config_c3, "c4": config_c4}


# ----------------------------------------------------------------------------
# The paper's other analytic systems (Sec. V-A, V-C, V-E) on scenes of the same kind.
# ----------------------------------------------------------------------------

def config_dubins(seed: int = 0, **over) -> Problem:
    """Dubins airplane, [0,10]^3, 30 boxes side U(0.5,2.5); B 4096, A 8, T 20, dt .05."""
    rng = np.random.default_rng([seed, 6])
    start = [1.0, 1.0, 1.0, 0.0, 0.0, 1.0]
    goal_c, goal_r = [9.0, 9.0, 9.0], 1.0
    scene = make_scene(rng, [0, 0, 0], [10, 10, 10], 30, (0.5, 2.5), 0, (0, 0), start[:3],
                       goal_c, goal_r)
    kw = dict(B=4096, A=8, T=20, dt=np.float32(0.05), n_cap=262144, cost_kind=COST_DURATION,
              seed=seed, name="dubins")
    kw.update(over)
    return build_problem(DUBINS, [0, 0, 0], [10, 10, 10], *scene, start, goal_c, goal_r, **kw)


def config_uni1(seed: int = 0, **over) -> Problem:
    """Unicycle 1, [0,10]^2, 40 square obstacles side U(0.5,1.2); B 1024, A 8, T 10, dt .1."""
    rng = np.random.default_rng([seed, 7])
    start = [1.0, 1.0, 0.0]
    goal_c, goal_r = [9.0, 9.0], 0.5
    scene = make_scene(rng, [0, 0], [10, 10], 40, (0.5, 1.2), 0, (0, 0), start[:2], goal_c,
                       goal_r, square=True)
    kw = dict(B=1024, A=8, T=10, dt=np.float32(0.1), n_cap=131072, cost_kind=COST_DURATION,
              seed=seed, name="uni1")
    kw.update(over)
    return build_problem(UNI1, [0, 0], [10, 10], *scene, start, goal_c, goal_r, **kw)


def config_uni2(seed: int = 0, **over) -> Problem:
    """Unicycle 2, [0,10]^2, 40 square obstacles side U(0.5,1.2); B 1024, A 8, T 10, dt .1."""
    rng = np.random.default_rng([seed, 8])
    start = [1.0, 1.0, 0.0, 0.0, 0.0]
    goal_c, goal_r = [9.0, 9.0], 0.5
    scene = make_scene(rng, [0, 0], [10, 10], 40, (0.5, 1.2), 0, (0, 0), start[:2], goal_c,
                       goal_r, square=True)
    kw = dict(B=1024, A=8, T=10, dt=np.float32(0.1), n_cap=131072, cost_kind=COST_DURATION,
              seed=seed, name="uni2")
    kw.update(over)
    return build_problem(UNI2, [0, 0], [10, 10], *scene, start, goal_c, goal_r, **kw)


def _no_obstacles(npos: int):
    return (np.zeros((0, npos)), np.zeros((0, npos)), np.zeros((0, npos)), np.zeros(0))


def config_acrobot(seed: int = 0, **over) -> Problem:
    """Acrobot swing-up: from hanging at rest to the upright configuration
    (shoulder pi, elbow 0) within 0.3 rad; configuration box [-2 pi, 2 pi]^2, no
    obstacles; B 1024, A 8, T 10, dt .02."""
    lo, hi = [-2 * math.pi, -2 * math.pi], [2 * math.pi, 2 * math.pi]
    kw = dict(B=1024, A=8, T=10, dt=np.float32(0.02), n_cap=131072, cost_kind=COST_DURATION,
              seed=seed, name="acrobot")
    kw.update(over)
    return build_problem(ACROBOT, lo, hi, *_no_obstacles(2), [0.0, 0.0, 0.0, 0.0],
                         [math.pi, 0.0], 0.3, **kw)


def config_cartpole(seed: int = 0, **over) -> Problem:
    """Cart-pole swing-up: from the pole hanging (angle pi) at rest to upright
    with the cart near the centre (within 0.3 of (0, 0)); cart in [-2.5, 2.5],
    angle in [-2 pi, 2 pi], no obstacles; B 1024, A 8, T 10, dt .02."""
    lo, hi = [-2.5, -2 * math.pi], [2.5, 2 * math.pi]
    kw = dict(B=1024, A=8, T=10, dt=np.float32(0.02), n_cap=131072, cost_kind=COST_DURATION,
              seed=seed, name="cartpole")
    kw.update(over)
    return build_problem(CARTPOLE, lo, hi, *_no_obstacles(2), [0.0, math.pi, 0.0, 0.0],
                         [0.0, 0.0], 0.3, **kw)


MORE_CONFIGS = {"dubins": config_dubins, "uni1": config_uni1, "uni2": config_uni2,
                "acrobot": config_acrobot, "cartpole": config_cartpole}

# Per-system planner settings used for the mixed batch.
_BATCH_SETTINGS = {
    DI3: dict(B=4096, A=8, T=20, dt=np.float32(0.05)),
    CAR: dict(B=8192, A=16, T=25, dt=np.float32(0.04)),
    QUAD: dict(B=8192, A=16, T=40, dt=np.float32(0.02)),
}


def config_c5(n_queries: int = 256, seed: int = 0, systems=(DI3, CAR, QUAD),
              settings: Optional[dict] = None) -> List[Problem]:
    """Mixed batch: query q uses systems[q % len(systems)], random start/goal/scene.

    Tree capacities are log-uniform in [4096, 262144] rounded up to 64, and at
    least one batch plus the root (B + 1, rounded up to 64); 10..60 obstacles per
    scene; start and goal at least 1 from the walls and at least half the
    workspace side apart.
    """
    out = []
    for q in range(n_queries):
        rng = np.random.default_rng([seed, 5, q])
        system = systems[q % len(systems)]
        side = 20.0 if system == CAR else 10.0
        D = 2 if system == CAR else 3
        ws_lo, ws_hi = [0.0] * D, [side] * D
        while True:
            s = rng.uniform(1.0, side - 1.0, size=D)
            g = rng.uniform(1.0, side - 1.0, size=D)
            if np.linalg.norm(g - s) >= 0.5 * side:
                break
        cap = int(math.exp(rng.uniform(math.log(4096), math.log(262144))))
        cap = (cap + 63) // 64 * 64
        n_obs = int(rng.integers(10, 61))
        goal_r = 1.0 if system != DI3 else 0.5
        if system == DI3:
            scene = make_scene(rng, ws_lo, ws_hi, n_obs, (0.5, 2.5), 0, (0, 0), s, g, goal_r)
        elif system == CAR:
            nb = (3 * n_obs) // 4
            scene = make_scene(rng, ws_lo, ws_hi, nb, (0.5, 2.0), n_obs - nb, (0.3, 1.0), s, g,
                               goal_r)
        else:
            scene = make_scene(rng, ws_lo, ws_hi, 0, (0, 0), n_obs, (0.3, 1.2), s, g, goal_r)
        t = system_table(system, ws_lo, ws_hi)
        x0 = np.zeros(t["d"])
        x0[:D] = s
        kw = dict(_BATCH_SETTINGS[system])
        if settings and system in settings:
            kw.update(settings[system])
        cap = max(cap, (kw["B"] + 1 + 63) // 64 * 64)
        kw.update(n_cap=cap, cost_kind=COST_DURATION, seed=seed, qid=q,
                  name=f"c5_q{q}_{SYSTEM_NAMES[system]}")
        out.append(build_problem(system, ws_lo, ws_hi, *scene, x0, g, goal_r, **kw))
    return out


@dataclasses.dataclass(frozen=True)
class RefineSettings:
    """Weights of the trajectory refinement objective (inputs, not arithmetic).

    Effort is measured from the middle of the control box (hover thrust for the
    quadrotor) in units of the box's half-range; beta = 20, delta = 0.1,
    w_c = w_g = 10, w_u = 1; 50 Adam steps of 1e-2 in the normalised controls.
    """
    w_u: float
    w_g: float
    w_c: float
    beta: float
    delta: float
    u_ref: tuple
    u_scale: tuple
    steps: int = 50
    lr: float = 1e-2


def refine_settings(prob: Problem, **over) -> RefineSettings:
    lo = np.asarray(prob.u_lo, np.float64)[:prob.m]
    hi = np.asarray(prob.u_hi, np.float64)[:prob.m]
    mid = [float(np.float32(v)) for v in 0.5 * (lo + hi)]
    half = [float(np.float32(v)) for v in 0.5 * (hi - lo)]
    kw = dict(w_u=1.0, w_g=10.0, w_c=10.0, beta=20.0, delta=0.1, u_ref=tuple(mid),
              u_scale=tuple(half))
    kw.update(over)
    return RefineSettings(**kw)
