"""Seeded synthetic inputs for the batched driving-physics step.

This module only *draws* inputs: road polylines, flat triangulated road
meshes, spawn/goal tables, per-surface friction classes, rain film depths,
vehicle parameter values and per-step actions.  It holds none of the
method's arithmetic (no physics, no friction mapping, no ride height, no
circle model); both the HIP path and the CPU oracle receive exactly these
arrays and derive everything else on their own.

Shapes follow the workloads the paper describes (Sec. "Per-scenario world
building", Sec. "Experimental Setup"): worlds are origin-centred, z-flattened
road layouts whose polylines are sampled at 0.5 m; lane centres carry type 2
and road edges types 15/16 (the Waymo codes the paper's reward section uses);
every world hosts up to its agent count of vehicles with start/goal pairs at
least 3 m apart.  The Waymo scenes themselves are not available, so these
procedural layouts stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# vehicle parameter values (configured values; derived quantities are not
# computed here)
# --------------------------------------------------------------------------

#: Configured vehicle: chassis/wheel/suspension values of the single-world
#: workload, actuation values of the paper's action-decoding table, and the
#: readings listed in the design notes for values the paper leaves open.
VEHICLE_DEFAULTS: dict = dict(
    mass=1500.0,
    inertia=(600.0, 2500.0, 2800.0),     # body (roll, pitch, yaw)
    wheel_radius=0.35,
    wheel_mass=20.0,
    wheel_inertia=0.0,                   # 0 -> solid disc
    susp_k=35000.0,
    susp_c=4000.0,
    susp_rest=0.30,
    mount=((1.3, 0.8, -0.20), (1.3, -0.8, -0.20),
           (-1.3, 0.8, -0.20), (-1.3, -0.8, -0.20)),   # FL, FR, RL, RR
    length=4.0,
    width=2.0,
    wheelbase=2.6,
    tau_drive=600.7,
    tau_brake_front=1090.5,
    tau_brake_rear=980.7,
    steer_kp=1839.5,
    steer_kd=110.5,
    steer_tau_max=1200.0,
    steer_inertia=0.6125,
    steer_max=0.5,
    c_kappa=12.0,
    c_alpha=10.0,
    v_eps=1.0,
    trail=0.03,
    yaw_damping=0.0,
    gravity=9.81,
    jacobi_iters=8,
    baumgarte=0.2,
    slop=0.01,
    max_episode_steps=1500,
    collision_warmup=24,
)

#: friction classes of the workloads (dry, wet, snow, ice)
MU_CLASSES = np.array([0.9, 0.6, 0.3, 0.1], dtype=np.float32)
#: friction classes of the tire-sampling workload (the four above plus the
#: hydroplaning floor's order of magnitude, for coverage of the network)
MU_SAMPLING = np.array([0.9, 0.6, 0.3, 0.1, 0.001], dtype=np.float32)

ROAD_LANE = 2
ROAD_EDGE_LEFT = 15
ROAD_EDGE_RIGHT = 16

LANE_W = 3.5
SPACING = 0.5
QUAD_LEN = 2.0


@dataclass
class Worlds:
    """CSR description of W worlds (all arrays host numpy)."""
    num_worlds: int
    agent_offsets: np.ndarray            # int32 [W+1]
    road_offsets: np.ndarray             # int32 [W+1]
    road_xy: np.ndarray                  # float32 [P,2]
    road_type: np.ndarray                # uint8 [P]
    tri_offsets: np.ndarray              # int32 [W+1]
    tri_verts: np.ndarray                # float32 [T,3,3]
    tri_surface: np.ndarray              # uint8 [T]
    num_surfaces: int
    mu_class: np.ndarray                 # float32 [W,S]
    film_mm: np.ndarray                  # float32 [W]
    pavement: np.ndarray                 # uint8 [W] (0 AC, 1 SMA, 2 OGFC)
    spawn_offsets: np.ndarray            # int32 [W+1]
    spawn: np.ndarray                    # float32 [E,5] x, y, yaw, goal_x, goal_y
    seed: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)
    road_dir: np.ndarray = None          # float32 [P,2] unit direction of each point's polyline

    @property
    def num_agents(self) -> int:
        return int(self.agent_offsets[-1])

    def world_slice(self, w0: int, w1: int) -> "Worlds":
        """Sub-batch of worlds [w0, w1) with re-based offsets."""
        def sub(off, *arrs):
            a, b = int(off[w0]), int(off[w1])
            return (off[w0:w1 + 1] - off[w0]).astype(np.int32), [x[a:b] for x in arrs]
        ao, _ = sub(self.agent_offsets)
        rdir = self.road_dir if self.road_dir is not None else np.zeros_like(self.road_xy)
        ro, (rxy, rty, rdr) = sub(self.road_offsets, self.road_xy, self.road_type, rdir)
        to, (tv, ts) = sub(self.tri_offsets, self.tri_verts, self.tri_surface)
        so, (sp,) = sub(self.spawn_offsets, self.spawn)
        return Worlds(w1 - w0, ao, ro, rxy.copy(), rty.copy(), to, tv.copy(), ts.copy(),
                      self.num_surfaces, self.mu_class[w0:w1].copy(),
                      self.film_mm[w0:w1].copy(), self.pavement[w0:w1].copy(),
                      so, sp.copy(), self.seed, self.name + f"[{w0}:{w1}]", dict(self.meta),
                      rdr.copy() if self.road_dir is not None else None)


# --------------------------------------------------------------------------
# road pieces
# --------------------------------------------------------------------------

class _Road:
    """Accumulates polyline points, triangles and lane records for one world."""

    def __init__(self):
        self.xy: list = []
        self.ty: list = []
        self.dr: list = []           # unit direction of each polyline point
        self.tris: list = []
        self.lanes: list = []        # (start_xy, unit travel dir, length)

    def straight(self, a, b, max_points=None):
        """One straight road piece from a to b: 4 lane centres (2 each way,
        3.5 m lanes) and 2 edges, sampled every 0.5 m, plus a flat mesh of
        2 m x 3.5 m lane quads.  Returns the number of points emitted."""
        a = np.asarray(a, np.float64)
        b = np.asarray(b, np.float64)
        length = float(np.linalg.norm(b - a))
        d = (b - a) / length
        left = np.array([-d[1], d[0]])
        n_pts = int(math.floor(length / SPACING + 1e-9)) + 1
        s = np.arange(n_pts) * SPACING
        emitted = 0
        # polylines: right edge, right lanes, left lanes, left edge; lane
        # centres point along their travel direction (right-hand traffic),
        # each edge along the lane next to it
        offsets = [(-2 * LANE_W, ROAD_EDGE_RIGHT), (-1.5 * LANE_W, ROAD_LANE),
                   (-0.5 * LANE_W, ROAD_LANE), (0.5 * LANE_W, ROAD_LANE),
                   (1.5 * LANE_W, ROAD_LANE), (2 * LANE_W, ROAD_EDGE_LEFT)]
        for off, ty in offsets:
            travel = d if off < 0 else -d
            pts = a[None, :] + s[:, None] * d[None, :] + off * left[None, :]
            if max_points is not None:
                room = max_points - emitted
                if room <= 0:
                    break
                pts = pts[:room]
            self.xy.append(pts)
            self.ty.append(np.full(len(pts), ty, np.uint8))
            self.dr.append(np.tile(travel, (len(pts), 1)))
            emitted += len(pts)
        # lane quads (flat, z = 0)
        n_q = int(math.floor(length / QUAD_LEN + 1e-9))
        for lane in range(4):
            o0 = (-2 + lane) * LANE_W
            o1 = o0 + LANE_W
            for k in range(n_q):
                s0, s1 = k * QUAD_LEN, (k + 1) * QUAD_LEN
                p00 = a + s0 * d + o0 * left
                p10 = a + s1 * d + o0 * left
                p11 = a + s1 * d + o1 * left
                p01 = a + s0 * d + o1 * left
                self.tris.append((p00, p10, p11))
                self.tris.append((p00, p11, p01))
        # lanes: right-hand traffic (right of the centreline travels along d)
        for off in (-1.5 * LANE_W, -0.5 * LANE_W):
            self.lanes.append((a + off * left, d.copy(), length))
        for off in (0.5 * LANE_W, 1.5 * LANE_W):
            self.lanes.append((b + off * left, -d, length))
        return emitted

    def arrays(self):
        xy = np.concatenate(self.xy).astype(np.float32) if self.xy else np.zeros((0, 2), np.float32)
        ty = np.concatenate(self.ty) if self.ty else np.zeros((0,), np.uint8)
        dr = np.concatenate(self.dr).astype(np.float32) if self.dr else np.zeros((0, 2), np.float32)
        if self.tris:
            t = np.array(self.tris, np.float64)                  # [T,3,2]
            tv = np.zeros((len(t), 3, 3), np.float32)
            tv[:, :, :2] = t
        else:
            tv = np.zeros((0, 3, 3), np.float32)
        return xy, ty, tv, dr


def _rot(v, ang):
    c, s = math.cos(ang), math.sin(ang)
    return np.array([c * v[0] - s * v[1], s * v[0] + c * v[1]])


def _spawn_table(rng, lanes, count, min_sep, headway=None, max_tries=20000, min_count=None):
    """Spawn entries (x, y, yaw, gx, gy) on lane centres.

    Entries are pairwise at least ``min_sep`` apart; with ``headway`` they are
    laid out lane by lane at gaps drawn from U[headway] so that consecutive
    entries form dense queues.  Goals lie 10..100 m ahead on the same lane
    (never past its end), hence always >= 3 m from the start."""
    out = []

    def ok(p, d):
        # same lane: at least min_sep apart; parallel neighbouring lanes:
        # 3 m (lanes are 3.5 m apart, wider than two circle radii); crossing
        # lanes: 4.6 m, enough that no two vehicle circles overlap
        for e in out:
            dx, dy = e[0] - p[0], e[1] - p[1]
            dist = math.hypot(dx, dy)
            ex, ey = math.cos(e[2]), math.sin(e[2])
            parallel = abs(ex * d[0] + ey * d[1]) > 0.99
            lateral = abs(d[0] * dy - d[1] * dx)
            need = (min_sep if lateral < 1.0 else 3.0) if parallel else 4.6
            if dist < need:
                return False
        return True

    def entry(lane, s):
        start, d, length = lane
        rem = length - s
        g = rng.uniform(10.0, min(100.0, rem))
        p = start + s * d
        q = start + (s + g) * d
        return (p[0], p[1], math.atan2(d[1], d[0]), q[0], q[1])

    if headway is not None:
        order = rng.permutation(len(lanes))
        for li in order:
            lane = lanes[li]
            s = rng.uniform(0.5, headway[1])
            while lane[2] - s >= 10.0:
                p = lane[0] + s * lane[1]
                if ok(p, lane[1]):
                    out.append(entry(lane, s))
                    if len(out) >= count:
                        return np.array(out, np.float32)
                s += rng.uniform(headway[0], headway[1])
        if len(out) < count:
            raise ValueError("not enough room for the requested spawn count")
        return np.array(out, np.float32)

    tries = 0
    while len(out) < count:
        tries += 1
        if tries > max_tries:
            if min_count is not None and len(out) >= min_count:
                break
            raise ValueError("could not place spawn entries")
        lane = lanes[rng.integers(len(lanes))]
        if lane[2] < 10.5:
            continue
        s = rng.uniform(0.0, lane[2] - 10.0)
        p = lane[0] + s * lane[1]
        if ok(p, lane[1]):
            out.append(entry(lane, s))
    return np.array(out, np.float32)


def _intersection(rng, arm_range=(38.0, 46.0)):
    """Two perpendicular 4-lane roads crossing at the origin, random heading."""
    road = _Road()
    phi = rng.uniform(0.0, 2 * math.pi)
    for k in range(2):
        arm = rng.uniform(*arm_range)
        d = _rot((1.0, 0.0), phi + k * math.pi / 2)
        road.straight(-arm * d, arm * d)
    return road


def _manhattan(rng, n_points, block=100.0):
    """A Manhattan grid of 100 m blocks grown edge by edge (nearest edges to
    the origin first) until exactly ``n_points`` polyline points exist."""
    road = _Road()
    edges = []
    R = 8
    for i in range(-R, R):
        for j in range(-R, R + 1):
            edges.append(((i * block, j * block), ((i + 1) * block, j * block)))
            edges.append(((j * block, i * block), (j * block, (i + 1) * block)))
    mid = np.array([[(a[0] + b[0]) / 2, (a[1] + b[1]) / 2] for a, b in edges])
    key = np.hypot(mid[:, 0], mid[:, 1]) + 1e-3 * np.arctan2(mid[:, 1], mid[:, 0])
    order = np.argsort(key, kind="stable")
    phi = rng.uniform(0.0, 2 * math.pi)
    shift = rng.uniform(-block / 2, block / 2, size=2)
    total = 0
    for e in order:
        if total >= n_points:
            break
        a, b = edges[e]
        a = _rot(np.array(a) + shift, phi)
        b = _rot(np.array(b) + shift, phi)
        total += road.straight(a, b, max_points=n_points - total)
    return road


def _pack(name, seed, roads, agents, spawns, mu_class, film, pavement):
    W = len(roads)
    xy, ty, tv, dr = zip(*[r.arrays() for r in roads])
    off = lambda sizes: np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    return Worlds(
        num_worlds=W,
        agent_offsets=off(agents),
        road_offsets=off([len(x) for x in xy]),
        road_xy=np.concatenate(xy).reshape(-1, 2).astype(np.float32),
        road_type=np.concatenate(ty).astype(np.uint8),
        tri_offsets=off([len(t) for t in tv]),
        tri_verts=np.concatenate(tv).reshape(-1, 3, 3).astype(np.float32),
        tri_surface=np.ones(sum(len(t) for t in tv), np.uint8),
        num_surfaces=mu_class.shape[1],
        mu_class=mu_class.astype(np.float32),
        film_mm=np.asarray(film, np.float32),
        pavement=np.asarray(pavement, np.uint8),
        spawn_offsets=off([len(s) for s in spawns]),
        spawn=np.concatenate(spawns).reshape(-1, 5).astype(np.float32),
        seed=int(seed),
        name=name,
        road_dir=np.concatenate(dr).reshape(-1, 2).astype(np.float32),
    )


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def flat_plane(n_agents=2, half=500.0, mu=0.9, spacing=20.0, goal_ahead=400.0, seed=0):
    """One world: a flat square of two road triangles, no polylines,
    ``n_agents`` vehicles side by side heading +x (single-world workload)."""
    tri = np.zeros((2, 3, 3), np.float32)
    tri[0, :, :2] = [(-half, -half), (half, -half), (half, half)]
    tri[1, :, :2] = [(-half, -half), (half, half), (-half, half)]
    ys = (np.arange(n_agents) - (n_agents - 1) / 2.0) * spacing
    spawn = np.array([(0.0, y, 0.0, goal_ahead, y) for y in ys], np.float32)
    return Worlds(
        num_worlds=1,
        agent_offsets=np.array([0, n_agents], np.int32),
        road_offsets=np.array([0, 0], np.int32),
        road_xy=np.zeros((0, 2), np.float32),
        road_type=np.zeros((0,), np.uint8),
        tri_offsets=np.array([0, 2], np.int32),
        tri_verts=tri,
        tri_surface=np.ones(2, np.uint8),
        num_surfaces=2,
        mu_class=np.full((1, 2), mu, np.float32),
        film_mm=np.zeros(1, np.float32),
        pavement=np.zeros(1, np.uint8),
        spawn_offsets=np.array([0, n_agents], np.int32),
        spawn=spawn,
        seed=seed,
        name="flat-plane 1x%d" % n_agents,
    )


def intersections(num_worlds=64, agents=8, seed=0, headway=None, min_sep=8.0,
                  spawn_factor=2, rain=False, name=None):
    """Worlds with one 4-way intersection of two 2+2-lane roads (~2k points),
    per-(world, surface) friction class, optional rain film depth."""
    rng = np.random.default_rng(seed)
    roads, spawns, film = [], [], []
    for w in range(num_worlds):
        road = _intersection(rng)
        roads.append(road)
        if headway is not None:
            spawns.append(_spawn_table(rng, road.lanes, agents, headway[0], headway=headway))
        else:
            spawns.append(_spawn_table(rng, road.lanes, spawn_factor * agents, min_sep))
        film.append(0.8 * rng.uniform(0.0, 1.0) if rain else 0.0)
    mu = MU_CLASSES[rng.integers(0, 4, size=(num_worlds, 2))]
    nm = name or f"intersections {num_worlds}x{agents}"
    return _pack(nm, seed, roads, [agents] * num_worlds, spawns, mu, film,
                 np.zeros(num_worlds, np.uint8))


def uneven_manhattan(num_worlds=256, agents=(4, 32), points=(1000, 20000), seed=0,
                     min_sep=8.0, spawn_factor=2, mean_agents=16):
    """Worlds with uneven agent counts U{agents} and road sizes U[points]: a
    Manhattan grid of the intersection cross-section grown to the drawn size."""
    rng = np.random.default_rng(seed)
    roads, spawns, counts = [], [], []
    # per-world agent counts span the whole range but total exactly
    # mean_agents * num_worlds slots (a plain uniform draw over 4..32 would
    # average 18, not 16): draw uniformly, then take single agents away from
    # randomly chosen worlds above the minimum until the total fits.
    a_w = rng.integers(agents[0], agents[1] + 1, size=num_worlds)
    target = int(mean_agents * num_worlds)
    while a_w.sum() > target:
        cand = np.nonzero(a_w > agents[0])[0]
        a_w[cand[rng.integers(len(cand))]] -= 1
    while a_w.sum() < target:
        cand = np.nonzero(a_w < agents[1])[0]
        a_w[cand[rng.integers(len(cand))]] += 1
    for w in range(num_worlds):
        a = int(a_w[w])
        p = int(rng.integers(points[0], points[1] + 1))
        road = _manhattan(rng, p)
        roads.append(road)
        spawns.append(_spawn_table(rng, road.lanes, spawn_factor * a, min_sep,
                                   max_tries=4000, min_count=a))
        counts.append(a)
    mu = MU_CLASSES[rng.integers(0, 4, size=(num_worlds, 2))]
    return _pack(f"uneven-manhattan {num_worlds}w", seed, roads, counts, spawns, mu,
                 np.zeros(num_worlds), np.zeros(num_worlds, np.uint8))


def tire_sampling(num_worlds=1024, agents=16, seed=0) -> Worlds:
    """The intersection worlds of the learned tire model's sample logging:
    friction per (world, surface) drawn from MU_SAMPLING."""
    w = intersections(num_worlds, agents, seed=seed, name=f"tire sampling {num_worlds}x{agents}")
    rng = np.random.default_rng([int(seed), 0x7E])
    w.mu_class = MU_SAMPLING[rng.integers(0, len(MU_SAMPLING), size=w.mu_class.shape)]
    return w


def speeds(seed: int, step: int, n: int, lo: float = 3.0, hi: float = 30.0) -> np.ndarray:
    """Seeded forward speeds U[lo, hi] m/s (re-initialisation of the sample logging)."""
    rng = np.random.default_rng([int(seed), int(step), 0x5B])
    return rng.uniform(lo, hi, n).astype(np.float32)


def workload(name: str, seed: int = 0) -> Worlds:
    """The named workloads (sizes as configured)."""
    if name == "plane1x2":
        return flat_plane(2, seed=seed)
    if name == "cross64x8":
        return intersections(64, 8, seed=seed)
    if name == "uneven256":
        return uneven_manhattan(256, seed=seed)
    if name == "cross1024x16":
        return intersections(1024, 16, seed=seed)
    if name == "dense4096x32":
        return intersections(4096, 32, seed=seed, headway=(6.0, 10.0), rain=True)
    raise KeyError(name)


#: physics timing of each workload: (control interval dt, substeps)
TIMING = {
    "plane1x2": (1.0 / 120.0, 1),
    "cross64x8": (1.0 / 60.0, 4),
    "uneven256": (1.0 / 30.0, 4),
    "cross1024x16": (1.0 / 30.0, 4),
    "dense4096x32": (1.0 / 30.0, 4),
}


def actions(seed: int, step: int, n: int, steer_max: float = 0.5) -> np.ndarray:
    """Seeded per-step actions: a_long ~ U[-1,1] (+drive / -brake), steer ~ U[-0.5,0.5] rad."""
    rng = np.random.default_rng([int(seed), int(step), 0x5F])
    a = np.empty((n, 2), np.float32)
    a[:, 0] = rng.uniform(-1.0, 1.0, n)
    a[:, 1] = rng.uniform(-steer_max, steer_max, n)
    return a


def mlp_params(sizes, seed: int):
    """Seeded Gaussian init N(0, 1/fan_in), zero biases; float32 masters."""
    rng = np.random.default_rng([int(seed), 0x317])
    Ws, bs = [], []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        Ws.append((rng.standard_normal((fo, fi)) / math.sqrt(fi)).astype(np.float32))
        bs.append(np.zeros(fo, np.float32))
    return Ws, bs
