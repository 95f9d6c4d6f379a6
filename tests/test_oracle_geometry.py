"""Pins for CollisionFree / state validity, NearestNeighbor and edge bookkeeping.

Validity (Sec. III feasibility, Sec. IV-A per-step checks): a point robot
must lie in the closed workspace, outside every closed obstacle, within the
state limits.  The reference's box test (max over axes of |p-c|-h) is checked
against a clamp-to-box distance, spheres against the plain distance, and both
on hypothesis-generated points and on exact boundary cases.  Nearest
neighbour is checked against scipy's KD-tree and on constructed ties.
"""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy.spatial import cKDTree

import oracle
from paper_2607_03987_amd import workloads as W


def scene_problem(system, boxes=(), spheres=(), **kw):
    D = 2 if system in (W.DI2, W.CAR) else 3
    ws_lo, ws_hi = [0.0] * D, [10.0] * D
    bc = [b[0] for b in boxes]
    bh = [b[1] for b in boxes]
    sc = [s[0] for s in spheres]
    sr = [s[1] for s in spheres]
    t = W.system_table(system, ws_lo, ws_hi)
    x0 = np.zeros(t["d"])
    x0[:D] = 0.5
    return W.build_problem(system, ws_lo, ws_hi, np.array(bc, np.float32).reshape(-1, D),
                           np.array(bh, np.float32).reshape(-1, D),
                           np.array(sc, np.float32).reshape(-1, D),
                           np.array(sr, np.float32).reshape(-1), x0, [9.5] * D, 0.4, **kw)


def f32(x):
    return float(np.float32(x))


def test_box_boundary_is_closed():
    p = scene_problem(W.DI2, boxes=[([5.0, 5.0], [1.0, 0.5])])
    cp = oracle.CProblem(p)
    assert not oracle.state_valid(cp, [6.0, 5.2, 0, 0])[0]       # on the face x = 6
    assert not oracle.state_valid(cp, [5.3, 5.5, 0, 0])[0]       # on the face y = 5.5
    assert not oracle.state_valid(cp, [6.0, 5.5, 0, 0])[0]       # corner
    assert oracle.state_valid(cp, [6.0 + 1e-9, 5.2, 0, 0])[0]
    assert oracle.state_valid(cp, [6.0, 5.5 + 1e-9, 0, 0])[0]
    v, near, margin = oracle.state_valid(cp, [6.0 + 2e-6, 5.2, 0, 0])
    assert v and near and margin == pytest.approx(2e-6)
    v, near, _ = oracle.state_valid(cp, [6.0 + 2e-5, 5.2, 0, 0])
    assert v and not near


def test_sphere_boundary_is_closed():
    p = scene_problem(W.DI3, spheres=[([5.0, 5.0, 5.0], 1.0)])
    cp = oracle.CProblem(p)
    assert not oracle.state_valid(cp, [6.0, 5.0, 5.0, 0, 0, 0])[0]
    assert oracle.state_valid(cp, [6.0 + 1e-9, 5.0, 5.0, 0, 0, 0])[0]
    assert not oracle.state_valid(cp, [5.0, 5.0, 5.0, 0, 0, 0])[0]


def test_workspace_closed_and_limits():
    p = scene_problem(W.DI2)
    cp = oracle.CProblem(p)
    assert oracle.state_valid(cp, [0.0, 10.0, 0, 0])[0]
    assert not oracle.state_valid(cp, [-1e-9, 5, 0, 0])[0]
    assert not oracle.state_valid(cp, [5, 10 + 1e-9, 0, 0])[0]
    # speed norm |v| <= 2 (closed)
    assert oracle.state_valid(cp, [5, 5, 1.2, 1.6])[0]
    assert not oracle.state_valid(cp, [5, 5, 1.2, 1.6 + 1e-6])[0]
    assert oracle.state_valid(cp, [5, 5, 1.99, 0.0])[0]
    assert not oracle.state_valid(cp, [5, 5, float("nan"), 0.0])[0]
    pc = oracle.CProblem(scene_problem(W.CAR))
    assert oracle.state_valid(pc, [5, 5, 100.0, 1.0, f32(0.6)])[0]   # heading unbounded
    assert not oracle.state_valid(pc, [5, 5, 0.0, 1.0001, 0.0])[0]
    assert not oracle.state_valid(pc, [5, 5, 0.0, 0.0, 0.61])[0]
    pq = oracle.CProblem(scene_problem(W.QUAD))
    x = np.array([5, 5, 5, 1.2, -1.2, 3.0, 3, -3, 3, 5, -5, 5], float)
    x[3], x[4] = f32(1.2), -f32(1.2)
    assert oracle.state_valid(pq, x)[0]
    for i, bump in [(3, 1e-6), (6, 1e-6), (11, 1e-6)]:
        y = x.copy()
        y[i] += bump
        assert not oracle.state_valid(pq, y)[0]


def _clamp_outside(p, c, h):
    q = np.clip(p, c - h, c + h)
    return float(np.linalg.norm(p - q)) > 0.0


coord = st.floats(0.0, 10.0, allow_nan=False, width=32)


@settings(max_examples=300, deadline=None)
@given(px=coord, py=coord, pz=coord,
       boxes=st.lists(st.tuples(coord, coord, coord, st.floats(0.0625, 3.0, width=32),
                                st.floats(0.0625, 3.0, width=32), st.floats(0.0625, 3.0, width=32)),
                      min_size=0, max_size=3),
       sph=st.lists(st.tuples(coord, coord, coord, st.floats(0.0625, 3.0, width=32)),
                    min_size=0, max_size=3))
def test_validity_matches_clamp_distance(px, py, pz, boxes, sph):
    bl = [((b[0], b[1], b[2]), (b[3], b[4], b[5])) for b in boxes]
    sl = [((s[0], s[1], s[2]), s[3]) for s in sph]
    p = scene_problem(W.DI3, boxes=bl, spheres=sl)
    cp = oracle.CProblem(p)
    pt = np.array([px, py, pz], np.float64)
    expect = True
    for c, h in zip(p.box_c.astype(np.float64), p.box_h.astype(np.float64)):
        expect &= _clamp_outside(pt, c, h)
    for c, r in zip(p.sph_c.astype(np.float64), p.sph_r.astype(np.float64)):
        expect &= float(np.linalg.norm(pt - c)) > r
    got = oracle.state_valid(cp, [px, py, pz, 0, 0, 0])[0]
    assert got == expect


def test_validity_dense_grid_tiny_scene():
    p = scene_problem(W.DI2, boxes=[([3.0, 3.0], [1.0, 2.0]), ([7.0, 6.0], [0.5, 0.5])],
                      spheres=[([5.0, 8.0], 1.25)])
    cp = oracle.CProblem(p)
    xs = np.linspace(0, 10, 81)
    free = 0
    for x in xs:
        for y in xs:
            got = oracle.state_valid(cp, [x, y, 0, 0])[0]
            inside = ((abs(x - 3) <= 1 and abs(y - 3) <= 2) or (abs(x - 7) <= .5 and abs(y - 6) <= .5)
                      or (x - 5) ** 2 + (y - 8) ** 2 <= 1.25 ** 2)
            assert got == (not inside), (x, y)
            free += got
    # grid area estimate of the free space: 100 - 8 - 1 - pi*1.25^2
    est = free / 81 ** 2 * 100
    assert abs(est - (100 - 9 - math.pi * 1.25 ** 2)) < 3.0


def test_nearest_matches_kdtree():
    rng = np.random.default_rng(2)
    for d in (4, 5, 6, 12):
        pts = rng.uniform(-5, 5, (3000, d))
        tree = cKDTree(pts)
        for q in rng.uniform(-5, 5, (50, d)):
            i, d2, d2b = oracle.nearest(pts, q)
            dist, j = tree.query(q, k=2)
            assert i == j[0]
            assert d2 == pytest.approx(dist[0] ** 2, rel=1e-12)
            assert d2b == pytest.approx(dist[1] ** 2, rel=1e-12)


def test_nearest_ties_go_to_lowest_index():
    pts = np.array([[1.0, 0, 0, 0], [0, 1.0, 0, 0], [-1.0, 0, 0, 0], [0, 0, 1.0, 0]])
    i, d2, d2b = oracle.nearest(pts, np.zeros(4))
    assert i == 0 and d2 == d2b == 1.0
    pts2 = np.vstack([np.full((3, 4), 7.0), [[0.5, 0, 0, 0]], [[0.5, 0, 0, 0]]])
    assert oracle.nearest(pts2, np.zeros(4))[0] == 3


def test_edge_checks_every_substep_not_between():
    # DI2 moving right at 2 m/s: sub-step positions 1.1, 1.2, ..., 2.0
    p = scene_problem(W.DI2, boxes=[([1.5, 5.0], [0.01, 1.0])], T=10, dt=np.float32(0.05))
    cp = oracle.CProblem(p)
    ok, xT, c, amb = oracle.edge(cp, [1.0, 5.0, 2.0, 0.0], 0.0, [0.0, 0.0])
    assert not ok                                   # the sub-step at x = 1.5 hits the slab
    # a slab strictly between two sub-steps is not detected (no continuous sweep)
    p2 = scene_problem(W.DI2, boxes=[([1.55, 5.0], [0.02, 1.0])], T=10, dt=np.float32(0.05))
    ok2, xT2, _, _ = oracle.edge(oracle.CProblem(p2), [1.0, 5.0, 2.0, 0.0], 0.0, [0.0, 0.0])
    assert ok2
    np.testing.assert_allclose(xT2, [1.0 + 2.0 * 10 * float(np.float32(0.05)), 5.0, 2.0, 0.0])
    # the start state is not re-checked: an edge may leave a region whose
    # boundary the parent sits on
    p3 = scene_problem(W.DI2, boxes=[([0.9, 5.0], [0.1, 1.0])], T=10, dt=np.float32(0.05))
    assert oracle.edge(oracle.CProblem(p3), [1.0, 5.0, 2.0, 0.0], 0.0, [0.0, 0.0])[0]


def test_edge_costs():
    dt = np.float32(0.05)
    p = scene_problem(W.DI2, T=10, dt=dt, cost_kind=W.COST_PATH_LENGTH)
    ok, xT, c, _ = oracle.edge(oracle.CProblem(p), [2.0, 2.0, 0.6, 0.8], 1.25, [0.0, 0.0])
    assert ok and c == pytest.approx(1.25 + 1.0 * 10 * float(dt), rel=1e-12)
    # accelerating from rest along x: length = 1/2 a t^2
    ok, xT, c, _ = oracle.edge(oracle.CProblem(p), [2.0, 2.0, 0.0, 0.0], 0.0, [1.0, 0.0])
    assert c == pytest.approx(0.5 * (10 * float(dt)) ** 2, rel=1e-12)
    pd = scene_problem(W.DI2, T=10, dt=dt, cost_kind=W.COST_DURATION)
    ok, xT, c, _ = oracle.edge(oracle.CProblem(pd), [2.0, 2.0, 0.6, 0.8], 3.0, [0.3, 0.1])
    assert c == 3.0 + 10 * float(dt)


def test_heuristic_kinds():
    for kind, ck, expect in [(W.H_ADMISSIBLE, W.COST_PATH_LENGTH, 5.0 - 0.4),
                             (W.H_ADMISSIBLE, W.COST_DURATION, (5.0 - 0.4) / 2.0),
                             (W.H_PAPER_LITERAL, W.COST_DURATION, 5.0),
                             (W.H_NONE, W.COST_DURATION, 0.0)]:
        p = scene_problem(W.DI2, h_kind=kind, cost_kind=ck)
        cp = oracle.CProblem(p)
        # goal centre (9.5, 9.5), radius 0.4; point at distance 5 (3-4-5)
        h = oracle.heuristic(cp, [9.5 - 3.0, 9.5 - 4.0, 0.0, 0.0])
        assert h == pytest.approx(expect, rel=1e-6)
    p = scene_problem(W.DI2)
    assert oracle.heuristic(oracle.CProblem(p), [9.6, 9.5, 0, 0]) == 0.0   # inside the goal
