"""Small world builders shared by the tests (inputs only, no physics)."""
import numpy as np

from paper_2605_08528_amd import inputs as I


def f32(x):
    return float(np.float32(x))


def params(**over):
    p = dict(I.VEHICLE_DEFAULTS)
    p.update(over)
    return p


def world(spawns, tris=None, road_xy=None, road_type=None, mu=0.9, mu_ground=None,
          seed=0, agents=None):
    """One world with explicit spawn entries [(x, y, yaw, gx, gy)], optional
    triangles [T,3,3] (surface 1) and road points [P,2]."""
    spawns = np.asarray(spawns, np.float32).reshape(-1, 5)
    A = len(spawns) if agents is None else agents
    if tris is None:
        half = 500.0
        tris = np.zeros((2, 3, 3), np.float32)
        tris[0, :, :2] = [(-half, -half), (half, -half), (half, half)]
        tris[1, :, :2] = [(-half, -half), (half, half), (-half, half)]
    tris = np.asarray(tris, np.float32).reshape(-1, 3, 3)
    road_xy = np.zeros((0, 2), np.float32) if road_xy is None else np.asarray(road_xy, np.float32).reshape(-1, 2)
    road_type = (np.full(len(road_xy), 2, np.uint8) if road_type is None
                 else np.asarray(road_type, np.uint8))
    mg = mu if mu_ground is None else mu_ground
    return I.Worlds(
        num_worlds=1,
        agent_offsets=np.array([0, A], np.int32),
        road_offsets=np.array([0, len(road_xy)], np.int32),
        road_xy=road_xy, road_type=road_type,
        tri_offsets=np.array([0, len(tris)], np.int32),
        tri_verts=tris, tri_surface=np.ones(len(tris), np.uint8),
        num_surfaces=2,
        mu_class=np.array([[mg, mu]], np.float32),
        film_mm=np.zeros(1, np.float32), pavement=np.zeros(1, np.uint8),
        spawn_offsets=np.array([0, len(spawns)], np.int32),
        spawn=spawns, seed=seed, name="test")


def yaw_quat(yaw):
    return np.cos(yaw / 2), 0.0, 0.0, np.sin(yaw / 2)
