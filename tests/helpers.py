"""Small world builders shared by the tests (inputs only, no physics), and
the check that explains a time-to-collision mismatch by a near-threshold
decision of the swept-circle definition."""
import math

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


def plain_worlds(num_worlds, agents, mu=0.9, half=40.0, seed=0):
    """``num_worlds`` worlds, each a flat square of two road triangles with
    no polylines and ``agents`` vehicles whose spawn entries sit on a 12 m
    grid (tests then place the vehicles through the state)."""
    W, A = int(num_worlds), int(agents)
    t = np.zeros((2, 3, 3), np.float32)
    t[0, :, :2] = [(-half, -half), (half, -half), (half, half)]
    t[1, :, :2] = [(-half, -half), (half, half), (-half, half)]
    g = int(np.ceil(np.sqrt(A)))
    ent = np.array([(12.0 * (a % g), 12.0 * (a // g), 0.0, 12.0 * (a % g) + 300.0, 12.0 * (a // g))
                    for a in range(A)], np.float32)
    off = lambda n: (np.arange(W + 1) * n).astype(np.int32)
    return I.Worlds(
        num_worlds=W, agent_offsets=off(A), road_offsets=np.zeros(W + 1, np.int32),
        road_xy=np.zeros((0, 2), np.float32), road_type=np.zeros(0, np.uint8),
        tri_offsets=off(2), tri_verts=np.tile(t, (W, 1, 1)), tri_surface=np.ones(2 * W, np.uint8),
        num_surfaces=2, mu_class=np.full((W, 2), mu, np.float32), film_mm=np.zeros(W, np.float32),
        pavement=np.zeros(W, np.uint8), spawn_offsets=off(A), spawn=np.tile(ent, (W, 1)),
        seed=seed, name=f"plain {W}x{A}")


# ------------------------------------------------------------ TTC decisions
#: a TTC entry may differ from the oracle's only where one of its decisions
#: sits this close (relative) to its threshold on the shared float state:
#: float32 rounding of positions (~1e-7 relative) and of the quadratic's
#: terms moves a decision only inside such a window, and a root whose
#: discriminant is this small relative to b^2 is ill-conditioned
TTC_MARGIN = 1e-4


def _heading(f, n):
    qw, qx, qy, qz = (float(v) for v in f[3:7, n])
    x, y = 1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy + qw * qz)
    L = math.hypot(x, y)
    return (1.0, 0.0) if L < 1e-12 else (x / L, y / L)


def ttc_explained(f, i, j, cr, cd, got, tol=1e-3):
    """Whether the time to collision ``got`` (s) of ego i towards neighbour
    j (global indices into the float64 state f [24][N]) is one that the
    swept-circle definition yields on this state up to a near-threshold
    decision: the FP64 value itself, the value with one decision within
    TTC_MARGIN of its threshold taken the other way (neighbour behind,
    circles touching, separating, no real root), or any value when the
    circle pair that sets the minimum has an ill-conditioned root.  Returns
    (explained, smallest margin)."""
    hix, hiy = _heading(f, i)
    hjx, hjy = _heading(f, j)
    dx, dy = float(f[0, j] - f[0, i]), float(f[1, j] - f[1, i])
    bx = hix * dx + hiy * dy
    m_behind = abs(bx) / max(math.hypot(dx, dy), 1e-12)
    dvx, dvy = float(f[7, j] - f[7, i]), float(f[8, j] - f[8, i])
    aq = dvx * dvx + dvy * dvy
    R2 = 4.0 * cr * cr
    pairs = []
    for a in range(3):
        for b in range(3):
            cx = (f[0, j] + (b - 1) * cd * hjx) - (f[0, i] + (a - 1) * cd * hix)
            cy = (f[1, j] + (b - 1) * cd * hjy) - (f[1, i] + (a - 1) * cd * hiy)
            c0 = cx * cx + cy * cy - R2
            bq = 2.0 * (cx * dvx + cy * dvy)
            disc = bq * bq - 4.0 * aq * c0
            m = {"touch": abs(c0) / R2,
                 "sep": abs(bq) / max(2.0 * math.hypot(cx, cy) * math.sqrt(aq), 1e-30),
                 "root": abs(disc) / max(bq * bq, 1e-30)}
            pairs.append((c0, bq, disc, m))

    def total(flip_behind=False, flip=(-1, "")):
        behind = (bx < 0.0) != flip_behind
        if behind:
            return 10.0, -1
        best, arg = 10.0, -1
        for p, (c0, bq, disc, _) in enumerate(pairs):
            touching, sep, miss = c0 <= 0.0, bq >= 0.0, disc < 0.0
            if flip[0] == p:
                touching ^= flip[1] == "touch"
                sep ^= flip[1] == "sep"
                miss ^= flip[1] == "root"
            if touching:
                t = 0.0
            elif sep or miss:
                continue
            else:
                t = 2.0 * c0 / (-bq + math.sqrt(max(disc, 0.0)))
            if t < best:
                best, arg = t, p
        return best, arg

    base, arg = total()
    cands = [base]
    margins = [m_behind] + [v for (_, _, _, m) in pairs for v in m.values()]
    if m_behind < TTC_MARGIN:
        cands.append(total(flip_behind=True)[0])
    for p, (_, _, _, m) in enumerate(pairs):
        for name, v in m.items():
            if v < TTC_MARGIN:
                cands.append(total(flip=(p, name))[0])
    if min(abs(got - c) for c in cands) <= tol:
        return True, min(margins)
    # the minimising pair's root itself is ill-conditioned
    if arg >= 0 and pairs[arg][0] > 0.0 and pairs[arg][3]["root"] < TTC_MARGIN:
        return True, pairs[arg][3]["root"]
    return False, min(margins)
