"""Pins of the oracle's dense shaping rewards and lane-forbidden event
(appendix "Reward Design Details": dense shaping rewards; Table "Reward
components used in all experiments"): known answers on hand-built roads,
one term at a time, plus the event and the reward sum inside the step."""
import math

import numpy as np
import pytest

from tests.helpers import f32, params, world

PX, PY, PZ, QW, QX, QY, QZ, VX, VY = range(9)
GX, GY = 20, 21
SINCE = 2
LANE, EDGE = 2, 15


@pytest.fixture(scope="module")
def O(oracle_mod):
    return oracle_mod


def road_world(points, types, dirs, goal=(500.0, 0.0), agents=None):
    """One world with the given road points (types, unit directions) and one
    vehicle (more with `agents`) whose pose the tests set."""
    sp = [(0.0, 0.0, 0.0, goal[0], goal[1])] + (agents or [])
    w = world(sp, road_xy=np.asarray(points, np.float32), road_type=np.asarray(types, np.uint8))
    w.road_dir = np.asarray(dirs, np.float32)
    return w


def place(o, i, x, y, yaw=0.0, vx=0.0, vy=0.0, goal=None):
    f, k = o.get_state()
    f[PX, i], f[PY, i] = x, y
    f[QW, i], f[QX, i], f[QY, i], f[QZ, i] = math.cos(yaw / 2), 0.0, 0.0, math.sin(yaw / 2)
    f[VX, i], f[VY, i] = vx, vy
    if goal is not None:
        f[GX, i], f[GY, i] = goal
    o.set_state(f, k)


def lane_along_x(y=0.0, n=81, x0=-20.0, dirx=1.0, ty=LANE):
    xs = x0 + 0.5 * np.arange(n)
    return [(x, y) for x in xs], [ty] * n, [(dirx, 0.0)] * n


def test_progress_along_the_lane_toward_the_goal(O):
    """Displacement projected on the nearest lane point's direction, the
    direction turned toward the goal, clamped to +-2 m, weight 2."""
    pts, ty, dr = lane_along_x()
    o = O.Oracle(road_world(pts, ty, dr), params())
    place(o, 0, 0.1, 0.0, goal=(100.0, 0.0))
    assert abs(o.shaping_terms(0, 0.7, 0.3)[0] - 2 * 0.7) < 1e-12
    assert abs(o.shaping_terms(0, 3.0, 0.0)[0] - 4.0) < 1e-12       # clamped
    assert abs(o.shaping_terms(0, -0.4, 0.0)[0] + 0.8) < 1e-12
    place(o, 0, 0.1, 0.0, goal=(-100.0, 0.0))                         # goal behind: the lane turns
    assert abs(o.shaping_terms(0, 0.7, 0.3)[0] + 1.4) < 1e-12


def test_lane_keeping_offset_and_heading(O):
    """q = exp(-(l / 1.75)^2) ((1 - 0.8) + 0.8 max(0, cos(psi - psi_lane))), weight 0.08."""
    pts, ty, dr = lane_along_x()
    o = O.Oracle(road_world(pts, ty, dr), params())
    for lat, yaw in ((0.0, 0.0), (1.0, 0.0), (-1.3, 0.0), (0.5, math.pi / 3), (0.5, math.pi * 0.9)):
        place(o, 0, 0.0, lat, yaw=yaw, goal=(100.0, 0.0))
        got = o.shaping_terms(0, 0.0, 0.0)[1]
        c = math.cos(np.float32(yaw / 2)) ** 2 - math.sin(np.float32(yaw / 2)) ** 2   # heading from the quaternion
        q = math.exp(-(f32(lat) / 1.75) ** 2) * (0.2 + 0.8 * max(0.0, c))
        assert abs(got - 0.08 * q) < 1e-6, (lat, yaw, got, 0.08 * q)


def test_off_road_lateral_and_distance(O):
    pts, ty, dr = lane_along_x()
    o = O.Oracle(road_world(pts, ty, dr), params())
    for lat, off in ((3.0, 0.0), (3.2, 0.0), (3.3, -0.5), (-3.4, -0.5)):
        place(o, 0, 0.0, lat, goal=(100.0, 0.0))
        assert o.shaping_terms(0, 0, 0)[2] == off, lat
    # the nearest lane point 6.5 m straight ahead (lateral 0): too far
    pts2, ty2, dr2 = [(6.5, 0.0)], [LANE], [(1.0, 0.0)]
    o2 = O.Oracle(road_world(pts2, ty2, dr2), params())
    place(o2, 0, 0.0, 0.0, goal=(100.0, 0.0))
    assert o2.shaping_terms(0, 0, 0)[2] == -0.5
    place(o2, 0, 1.0, 0.0, goal=(100.0, 0.0))          # 5.5 m: on the road
    assert o2.shaping_terms(0, 0, 0)[2] == 0.0
    # no lane point at all (only edges): off-road, no progress or lane term
    o3 = O.Oracle(road_world(pts2, [EDGE], dr2), params())
    place(o3, 0, 0.0, 0.0, goal=(100.0, 0.0))
    t = o3.shaping_terms(0, 1.0, 0.0)
    assert t[0] == 0.0 and t[1] == 0.0 and t[2] == -0.5


def test_idle_below_one_metre_per_second(O):
    pts, ty, dr = lane_along_x()
    o = O.Oracle(road_world(pts, ty, dr), params())
    for v, pen in ((0.0, -0.05), (0.9, -0.05), (0.7 * math.sqrt(2) * 0.999, -0.05), (1.1, 0.0)):
        place(o, 0, 0.0, 0.0, vx=v * math.cos(0.3), vy=v * math.sin(0.3), goal=(100.0, 0.0))
        assert o.shaping_terms(0, 0, 0)[3] == pen, v


def test_vehicle_ttc_penalty(O):
    """Another vehicle 20 m ahead, closing at 8 m/s head-on: the front
    circles touch after (20 - 2 d - 2 r) / 8 s; penalty min(0.1 / max(tau,
    0.5), 0.35); alone: tau = 10 s -> 0.01."""
    pts, ty, dr = lane_along_x()
    o = O.Oracle(road_world(pts, ty, dr, agents=[(20.0, 0.0, math.pi, -100.0, 0.0)]), params())
    place(o, 0, 0.0, 0.0, vx=8.0, goal=(100.0, 0.0))
    place(o, 1, 20.0, 0.0, yaw=math.pi, vx=0.0, goal=(-100.0, 0.0))
    cr, cd = O.circle_model(params())
    tau = (20.0 - 2 * cd - 2 * cr) / 8.0
    assert abs(o.shaping_terms(0, 0, 0)[4] + min(0.1 / max(tau, 0.5), 0.35)) < 1e-6
    place(o, 1, 9.0, 0.0, yaw=math.pi, vx=0.0, goal=(-100.0, 0.0))       # 0.5 s floor, then the 0.35 cap
    tau = (9.0 - 2 * cd - 2 * cr) / 8.0
    assert abs(o.shaping_terms(0, 0, 0)[4] + min(0.1 / max(tau, 0.5), 0.35)) < 1e-6
    o2 = O.Oracle(road_world(pts, ty, dr), params())
    place(o2, 0, 0.0, 0.0, vx=8.0, goal=(100.0, 0.0))
    assert abs(o2.shaping_terms(0, 0, 0)[4] + 0.01) < 1e-12


def test_road_edge_ttc_ahead_in_the_corridor(O):
    """An edge point 10 m ahead on the vehicle's line at 5 m/s: the front
    circle (d + r ahead of the centre) reaches it after (10 - d - r) / 5 s;
    penalty min(0.07 / max(tau, 0.5), 0.4).  Edge points behind, beside the
    corridor (|lateral| > W / 2 + r) or a vehicle standing still give 0."""
    cr, cd = O.circle_model(params())
    pts = [(10.0, 0.0), (-5.0, 0.0), (3.0, 2.2)]
    o = O.Oracle(road_world(pts, [EDGE] * 3, [(0.0, 1.0)] * 3), params())
    place(o, 0, 0.0, 0.0, vx=5.0, goal=(100.0, 0.0))
    tau = (10.0 - cd - cr) / 5.0
    assert abs(o.shaping_terms(0, 0, 0)[5] + min(0.07 / max(tau, 0.5), 0.4)) < 1e-6
    place(o, 0, 0.0, 0.0, vx=0.0, goal=(100.0, 0.0))
    assert o.shaping_terms(0, 0, 0)[5] == 0.0
    place(o, 0, 0.0, 0.0, vx=-5.0, goal=(100.0, 0.0))
    assert o.shaping_terms(0, 0, 0)[5] == 0.0
    o2 = O.Oracle(road_world([(3.0, 2.2)], [EDGE], [(1.0, 0.0)]), params())
    place(o2, 0, 0.0, 0.0, vx=5.0, goal=(100.0, 0.0))
    assert 2.2 > 1.0 + cr and o2.shaping_terms(0, 0, 0)[5] == 0.0
    o3 = O.Oracle(road_world([(3.0, 2.0)], [EDGE], [(1.0, 0.0)]), params())
    place(o3, 0, 0.0, 0.0, vx=5.0, goal=(100.0, 0.0))        # inside the corridor, 3 m ahead
    assert abs(o3.shaping_terms(0, 0, 0)[5] + min(0.07 / max((3.0 - cd - cr) / 5.0, 0.5), 0.4)) < 1e-6


@pytest.mark.parametrize("dist,hit", [(1.0, True), (1.09, True), (1.12, False), (1.3, False)])
def test_lane_forbidden_circle_against_edge_segment(O, dist, hit):
    """An edge segment (0.5 m, centred on its point, along x) at lateral
    distance `dist` from the vehicle's centre line: the circles (r = 1.1 m)
    overlap it iff dist < r; lane points never count."""
    o = O.Oracle(road_world([(0.3, dist)], [EDGE], [(1.0, 0.0)]), params())
    place(o, 0, 0.0, 0.0, goal=(100.0, 0.0))
    assert o.lane_forbidden(0) == hit
    o2 = O.Oracle(road_world([(0.3, dist)], [LANE], [(1.0, 0.0)]), params())
    place(o2, 0, 0.0, 0.0, goal=(100.0, 0.0))
    assert not o2.lane_forbidden(0)


def test_lane_forbidden_segment_ends(O):
    """The segment ends 0.25 m from its point: an edge point 1.0 m beyond
    the front circle's centre along the heading is 0.75 m from the circle's
    centre at its near end (overlap), one 1.4 m beyond is 1.15 m (none)."""
    cr, cd = O.circle_model(params())
    for ahead, hit in ((1.0, True), (1.4, False)):
        o = O.Oracle(road_world([(cd + ahead, 0.0)], [EDGE], [(1.0, 0.0)]), params())
        place(o, 0, 0.0, 0.0, goal=(100.0, 0.0))
        assert o.lane_forbidden(0) == hit, ahead


def test_step_rewards_with_shaping(O):
    """Inside the step: an agent touching a road edge at the start of the
    control step terminates with -20 (and is parked); another agent on its
    lane receives the sum of the six dense terms of its new pose."""
    pts, ty, dr = lane_along_x(n=121, x0=-30.0)
    pts = pts + [(-10.0, 30.0 + 0.9)]
    ty = ty + [EDGE]
    dr = dr + [(1.0, 0.0)]
    o = O.Oracle(road_world(pts, ty, dr, agents=[(-10.0, 30.0, 0.0, 100.0, 30.0)]), params())
    o.set_shaping(True)
    place(o, 0, 0.0, 0.3, vx=6.0, goal=(100.0, 0.0))
    place(o, 1, -10.0, 30.0, vx=3.0, goal=(100.0, 30.0))
    f, k = o.get_state()
    f[13:17] = f[VX] / 0.35
    k[SINCE] = 100
    o.set_state(f, k)
    assert o.lane_forbidden(1) and not o.lane_forbidden(0)
    x0, y0 = f[PX, 0], f[PY, 0]
    rew, done, ev = o.step(np.zeros((2, 2), np.float32), f32(1 / 30), 4)
    assert ev[1] & O.EV_LANE_FORBIDDEN and done[1] == 1 and rew[1] == -20.0
    f2, k2 = o.get_state()
    assert k2[0, 1] == 0 and f2[PX, 1] == 1000.0
    assert not ev[0] & O.EV_LANE_FORBIDDEN and done[0] == 0
    terms = o.shaping_terms(0, f2[PX, 0] - x0, f2[PY, 0] - y0)
    assert abs(rew[0] - np.float32(terms.sum())) < 1e-6
    assert terms[0] > 0.0 and terms[1] > 0.0 and terms[2] == 0.0
    # shaping off: the same step gives the sparse rewards only
    o.set_shaping(False)
    o.set_state(f, k)
    rew, done, ev = o.step(np.zeros((2, 2), np.float32), f32(1 / 30), 4)
    assert rew[0] == 0.0 and rew[1] == 0.0 and not ev[1] & O.EV_LANE_FORBIDDEN
