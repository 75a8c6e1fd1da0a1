"""TEST INFRASTRUCTURE ONLY: ctypes binding of the FP64 CPU oracle.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this module.  It wraps ``sf_oracle.c`` (plain brute-force C,
double precision) and knows nothing about the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SF_ORACLE_LIBRARY names another build (the AddressSanitizer build)
LIB_PATH = os.environ.get("SF_ORACLE_LIBRARY") or os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "sf_oracle.c")

NF, NK, NDYN = 24, 4, 19
FIELDS = ["px", "py", "pz", "qw", "qx", "qy", "qz", "vx", "vy", "vz", "wx", "wy", "wz",
          "om0", "om1", "om2", "om3", "th", "thd", "mu", "gx", "gy", "sx", "sy"]
IFIELDS = ["active", "ep_step", "since", "episode"]
EV_GOAL, EV_COLLISION, EV_CRASH, EV_TIMEOUT, EV_NUMERIC, EV_NAN_ACTION = 1, 2, 4, 8, 16, 32
EV_LANE_FORBIDDEN = 128
SUR_IN, SUR_HID, SAMPLE = 16, 128, 20
SUR_SIZES = [16, 128, 128, 128, 3]
SUR_PARAMS = 16 * 128 + 128 + 2 * (128 * 128 + 128) + 3 * 128 + 3
# the paper's observation and the late-fusion actor-critic
FULL_EGO, FULL_ROAD_K, FULL_NEIGH_K = 11, 350, 24
FULL_DIM = FULL_EGO + 5 * FULL_ROAD_K + 7 * FULL_NEIGH_K
AC_BODY = (11 * 64 + 64 + 64 * 64 + 64 + 5 * 96 + 96 + 96 * 96 + 96 + 7 * 96 + 96 + 96 * 96 + 96
           + 256 * 128 + 128 + 128 * 64 + 64)
AC_PARAMS = 2 * AC_BODY + 3 * 64 + 3 + 3 + 64 + 1


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (gcc, -O2, OpenMP);
    sanitize=True builds ``oracle/liboracle_asan.so`` with AddressSanitizer
    (load it with gcc's libasan preloaded)."""
    out = os.path.join(HERE, "liboracle_asan.so") if sanitize else os.path.join(HERE, "liboracle.so")
    san = ["-fsanitize=address", "-fno-omit-frame-pointer", "-g"] if sanitize else []
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-D_GNU_SOURCE", *san,
           "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


class OrParams(C.Structure):
    _fields_ = [
        ("mass", C.c_double), ("inertia", C.c_double * 3),
        ("wheel_radius", C.c_double), ("wheel_mass", C.c_double), ("wheel_inertia", C.c_double),
        ("susp_k", C.c_double), ("susp_c", C.c_double), ("susp_rest", C.c_double),
        ("mount", (C.c_double * 3) * 4),
        ("length", C.c_double), ("width", C.c_double), ("wheelbase", C.c_double),
        ("tau_drive", C.c_double), ("tau_brake_front", C.c_double), ("tau_brake_rear", C.c_double),
        ("steer_kp", C.c_double), ("steer_kd", C.c_double), ("steer_tau_max", C.c_double),
        ("steer_inertia", C.c_double), ("steer_max", C.c_double),
        ("c_kappa", C.c_double), ("c_alpha", C.c_double), ("v_eps", C.c_double),
        ("trail", C.c_double), ("yaw_damping", C.c_double), ("gravity", C.c_double),
        ("jacobi_iters", C.c_int), ("baumgarte", C.c_double), ("slop", C.c_double),
        ("max_episode_steps", C.c_int), ("collision_warmup", C.c_int),
        ("invincible", C.c_int), ("auto_reset", C.c_int),
    ]


class OrWorld(C.Structure):
    _fields_ = [
        ("num_worlds", C.c_int),
        ("agent_offsets", C.c_void_p),
        ("road_offsets", C.c_void_p), ("road_xy", C.c_void_p), ("road_type", C.c_void_p),
        ("tri_offsets", C.c_void_p), ("tri_verts", C.c_void_p), ("tri_surface", C.c_void_p),
        ("num_surfaces", C.c_int), ("mu_class", C.c_void_p),
        ("film_mm", C.c_void_p), ("pavement", C.c_void_p),
        ("spawn_offsets", C.c_void_p), ("spawn", C.c_void_p),
        ("seed", C.c_uint64),
        ("road_dir", C.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.c_int
        L.or_create.restype = vp
        L.or_create.argtypes = [C.POINTER(OrWorld), C.POINTER(OrParams)]
        L.or_destroy.argtypes = [vp]
        L.or_num_agents.argtypes = [vp]
        L.or_get_state.argtypes = [vp, vp, vp]
        L.or_set_state.argtypes = [vp, vp, vp]
        L.or_get_mu.argtypes = [vp, vp]
        L.or_step.argtypes = [vp, vp, C.c_double, ip, vp, vp, vp, vp, vp, ip]
        L.or_observe.argtypes = [vp, vp]
        L.or_reset.argtypes = [vp, vp]
        L.or_detect_pairs.argtypes = [vp, ip, vp, ip]
        L.or_detect_pairs.restype = ip
        L.or_events.argtypes = [vp, vp, vp]
        L.or_knn_road.argtypes = [vp, ip, vp]
        L.or_knn_neigh.argtypes = [vp, ip, vp]
        L.or_raycast.argtypes = [vp, ip, ip, dp, vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.or_raycast.restype = ip
        L.or_weather_mu.restype = C.c_double
        L.or_weather_mu.argtypes = [C.c_double, C.c_double, ip]
        L.or_set_bf16.argtypes = [ip]
        L.or_circle_model.argtypes = [C.POINTER(OrParams), dp, dp]
        L.or_mlp_forward.argtypes = [ip, vp, vp, vp, ip, ip, vp, vp]
        L.or_policy.argtypes = [ip, vp, vp, vp, C.c_double, vp]
        L.or_mlp_mse_grad.argtypes = [ip, vp, vp, vp, ip, vp, vp, vp, vp, vp]
        L.or_mlp_mse_grad.restype = C.c_double
        L.or_adam.argtypes = [ip, vp, vp, vp, vp, ip, C.c_double, C.c_double, C.c_double, C.c_double]
        L.or_tire.argtypes = [C.POINTER(OrParams)] + [C.c_double] * 8 + [dp] * 4
        L.or_set_threads.argtypes = [ip]
        L.or_set_surrogate.argtypes = [vp, vp, vp, vp, ip]
        L.or_surrogate_counts.argtypes = [vp, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]
        L.or_record_samples.argtypes = [vp, vp]
        L.or_set_dynamics.argtypes = [vp, ip]
        L.or_observe_full.argtypes = [vp, vp, vp]
        L.or_set_shaping.argtypes = [vp, ip]
        L.or_shaping_terms.argtypes = [vp, ip, C.c_double, C.c_double, vp]
        L.or_lane_forbidden.argtypes = [vp, ip]
        L.or_lane_forbidden.restype = ip
        L.or_road_within.argtypes = [vp, ip, ip, vp]
        L.or_road_within.restype = ip
        L.or_knn_neigh_k.argtypes = [vp, ip, ip, vp]
        L.or_actor_critic.argtypes = [vp, ip, vp, vp, vp, vp]
        L.or_set_tri_friction.argtypes = [vp, vp]
        L.or_set_tri_friction.restype = ip
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def make_params(prm: dict, invincible=False, auto_reset=False) -> OrParams:
    p = OrParams()
    for name, _ in OrParams._fields_:
        if name in ("invincible", "auto_reset"):
            continue
        v = prm[name]
        if name == "inertia":
            for k in range(3):
                p.inertia[k] = float(np.float32(v[k]))
        elif name == "mount":
            for r in range(4):
                for c in range(3):
                    p.mount[r][c] = float(np.float32(v[r][c]))
        elif name in ("jacobi_iters", "max_episode_steps", "collision_warmup"):
            setattr(p, name, int(v))
        else:
            # the configured values reach both implementations as float32
            setattr(p, name, float(np.float32(v)))
    p.invincible = int(invincible)
    p.auto_reset = int(auto_reset)
    return p


def weather_mu(mu_class: float, film_mm: float, pavement: int = 0) -> float:
    return lib().or_weather_mu(float(mu_class), float(film_mm), int(pavement))


def set_bf16(on: bool) -> None:
    lib().or_set_bf16(int(bool(on)))


def circle_model(prm: dict):
    r, d = C.c_double(), C.c_double()
    lib().or_circle_model(C.byref(make_params(prm)), C.byref(r), C.byref(d))
    return r.value, d.value


def tire(prm: dict, h, Fz, mu, vx, vy, omega, tau_d, tau_b):
    out = [C.c_double() for _ in range(4)]
    lib().or_tire(C.byref(make_params(prm)), h, Fz, mu, vx, vy, omega, tau_d, tau_b,
                  *[C.byref(o) for o in out])
    return tuple(o.value for o in out)


class Oracle:
    """FP64 brute-force simulator with the same logical calls as the library."""

    def __init__(self, worlds, params: dict, invincible=False, auto_reset=False, threads=None):
        L = lib()
        if threads:
            L.or_set_threads(int(threads))
        self.worlds = worlds
        self.params = dict(params)
        self._keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return _ptr(a)

        w = OrWorld()
        w.num_worlds = worlds.num_worlds
        w.agent_offsets = arr(worlds.agent_offsets, np.int32)
        w.road_offsets = arr(worlds.road_offsets, np.int32)
        w.road_xy = arr(worlds.road_xy, np.float32)
        w.road_type = arr(worlds.road_type, np.uint8)
        w.tri_offsets = arr(worlds.tri_offsets, np.int32)
        w.tri_verts = arr(worlds.tri_verts, np.float32)
        w.tri_surface = arr(worlds.tri_surface, np.uint8)
        w.num_surfaces = worlds.num_surfaces
        w.mu_class = arr(worlds.mu_class, np.float32)
        w.film_mm = arr(worlds.film_mm, np.float32)
        w.pavement = arr(worlds.pavement, np.uint8)
        w.spawn_offsets = arr(worlds.spawn_offsets, np.int32)
        w.spawn = arr(worlds.spawn, np.float32)
        w.seed = int(worlds.seed)
        if getattr(worlds, "road_dir", None) is not None:
            w.road_dir = arr(worlds.road_dir, np.float32)
        self._p = make_params(params, invincible, auto_reset)
        self.h = L.or_create(C.byref(w), C.byref(self._p))
        self._keep = []
        self.N = L.or_num_agents(self.h)
        self.W = worlds.num_worlds

    def close(self):
        if self.h:
            lib().or_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # state --------------------------------------------------------------
    def get_state(self):
        f = np.zeros((NF, self.N), np.float64)
        k = np.zeros((NK, self.N), np.int32)
        lib().or_get_state(self.h, _ptr(f), _ptr(k))
        return f, k

    def set_state(self, f, k):
        f = np.ascontiguousarray(f, np.float64)
        k = np.ascontiguousarray(k, np.int32)
        lib().or_set_state(self.h, _ptr(f), _ptr(k))

    def mu_table(self):
        mu = np.zeros((self.W, self.worlds.num_surfaces), np.float64)
        lib().or_get_mu(self.h, _ptr(mu))
        return mu

    # calls --------------------------------------------------------------
    def step(self, actions, dt, substeps, record_pairs=False, pair_cap=None):
        a = np.ascontiguousarray(actions, np.float32).reshape(self.N, 2)
        rew = np.zeros(self.N, np.float32)
        done = np.zeros(self.N, np.uint8)
        ev = np.zeros(self.N, np.uint8)
        rec = cnt = None
        if record_pairs:
            amax = int(np.diff(self.worlds.agent_offsets).max()) if self.W else 0
            pair_cap = pair_cap or max(1, amax * (amax - 1) // 2)
            rec = np.zeros((substeps, self.W, pair_cap), np.uint32)
            cnt = np.zeros((substeps, self.W), np.int32)
        lib().or_step(self.h, _ptr(a), float(dt), int(substeps), _ptr(rew), _ptr(done), _ptr(ev),
                      _ptr(rec), _ptr(cnt), int(pair_cap or 0))
        if record_pairs:
            return rew, done, ev, (rec, cnt)
        return rew, done, ev

    def observe(self):
        obs = np.zeros((self.N, 256), np.float32)
        lib().or_observe(self.h, _ptr(obs))
        return obs

    def reset(self, mask):
        m = np.ascontiguousarray(mask, np.uint8)
        lib().or_reset(self.h, _ptr(m))

    def set_shaping(self, on: bool):
        """Dense shaping rewards and the lane-forbidden event on or off."""
        lib().or_set_shaping(self.h, int(bool(on)))

    def shaping_terms(self, i, dx, dy):
        """(progress, lane keeping, off-road, idle, vehicle TTC, road-edge TTC)
        of agent i on the current pose after a displacement (dx, dy)."""
        t = np.zeros(6, np.float64)
        lib().or_shaping_terms(self.h, int(i), float(dx), float(dy), _ptr(t))
        return t

    def lane_forbidden(self, i) -> bool:
        return bool(lib().or_lane_forbidden(self.h, int(i)))

    def observe_full(self):
        """The paper's observation [N, 1929] and valid (road, neighbour) slot counts [N, 2]."""
        obs = np.zeros((self.N, FULL_DIM), np.float32)
        cnt = np.zeros((self.N, 2), np.int32)
        lib().or_observe_full(self.h, _ptr(obs), _ptr(cnt))
        return obs, cnt

    def road_within(self, i, K=FULL_ROAD_K):
        out = np.zeros(K, np.int32)
        n = lib().or_road_within(self.h, int(i), int(K), _ptr(out))
        return out, n

    def knn_neigh_k(self, i, K=FULL_NEIGH_K):
        out = np.zeros(K, np.int32)
        lib().or_knn_neigh_k(self.h, int(i), int(K), _ptr(out))
        return out

    def set_dynamics(self, mode: str):
        """'physics' (the articulated vehicle) or 'bicycle' (kinematic model)."""
        lib().or_set_dynamics(self.h, {"physics": 0, "bicycle": 1}[mode])

    def set_tri_friction(self, scale):
        """Friction factor per road triangle [T] (None clears it)."""
        if scale is None:
            lib().or_set_tri_friction(self.h, None)
            return
        self._tri_mu = np.ascontiguousarray(scale, np.float32)
        if lib().or_set_tri_friction(self.h, _ptr(self._tri_mu)) != 0:
            raise ValueError("triangle friction factors must be finite and >= 0")

    def set_surrogate(self, params, env_lo, env_hi, enable=True):
        self._sur = [np.ascontiguousarray(params, np.float32), np.ascontiguousarray(env_lo, np.float32),
                     np.ascontiguousarray(env_hi, np.float32)]
        lib().or_set_surrogate(self.h, *[_ptr(a) for a in self._sur], int(enable))

    def surrogate_counts(self):
        u, f = C.c_longlong(), C.c_longlong()
        lib().or_surrogate_counts(self.h, C.byref(u), C.byref(f))
        return u.value, f.value

    def record_samples(self, on=True):
        """Start recording the last substep's per-wheel surrogate samples."""
        if on:
            self._rec = np.zeros((self.N, 4, SAMPLE), np.float32)
            lib().or_record_samples(self.h, _ptr(self._rec))
        else:
            lib().or_record_samples(self.h, None)
            self._rec = None

    def samples(self):
        return self._rec.copy()

    def detect_pairs(self, world):
        a = int(self.worlds.agent_offsets[world + 1] - self.worlds.agent_offsets[world])
        cap = max(1, a * (a - 1) // 2)
        out = np.zeros(cap, np.uint32)
        n = lib().or_detect_pairs(self.h, int(world), _ptr(out), cap)
        return out[:n].copy()

    def events(self, collided):
        c = np.ascontiguousarray(collided, np.uint8)
        ev = np.zeros(self.N, np.uint8)
        lib().or_events(self.h, _ptr(c), _ptr(ev))
        return ev

    def knn_road(self, agent):
        out = np.zeros(64, np.int32)
        lib().or_knn_road(self.h, int(agent), _ptr(out))
        return out

    def knn_neigh(self, agent):
        out = np.zeros(8, np.int32)
        lib().or_knn_neigh(self.h, int(agent), _ptr(out))
        return out

    def raycast(self, agent, wheel):
        t = C.c_double()
        n = np.zeros(3, np.float64)
        s, tri = C.c_int(), C.c_int()
        hit = lib().or_raycast(self.h, int(agent), int(wheel), C.byref(t), _ptr(n), C.byref(s), C.byref(tri))
        return bool(hit), t.value, n, s.value, tri.value


def _layer_ptrs(Ws, bs):
    Wc = [np.ascontiguousarray(w, np.float32) for w in Ws]
    bc = [np.ascontiguousarray(b, np.float32) for b in bs]
    Wp = (C.c_void_p * len(Wc))(*[_ptr(w) for w in Wc])
    bp = (C.c_void_p * len(bc))(*[_ptr(b) for b in bc])
    return Wc, bc, Wp, bp


def mlp_forward(Ws, bs, x, act="relu"):
    sizes = np.array([Ws[0].shape[1]] + [w.shape[0] for w in Ws], np.int32)
    Wc, bc, Wp, bp = _layer_ptrs(Ws, bs)
    x = np.ascontiguousarray(x, np.float32)
    y = np.zeros((x.shape[0], sizes[-1]), np.float64)
    lib().or_mlp_forward(len(Ws), _ptr(sizes), Wp, bp, 0 if act == "elu" else 1, x.shape[0], _ptr(x), _ptr(y))
    return y


def policy(Ws, bs, obs, steer_max=0.5):
    Wc, bc, Wp, bp = _layer_ptrs(Ws, bs)
    obs = np.ascontiguousarray(obs, np.float32)
    act = np.zeros((obs.shape[0], 2), np.float64)
    lib().or_policy(obs.shape[0], _ptr(obs), Wp, bp, float(steer_max), _ptr(act))
    return act


def force_weights(target):
    """Training weight of a tire-model sample: 1 / max(|(F_x, F_y)|, 0.05)^2
    of its targets (in units of mu F_z), the squared denominator of the
    relative force error, so that the weighted squared error is the squared
    relative error that metric measures."""
    t = np.asarray(target, np.float64)
    return 1.0 / np.maximum(np.hypot(t[:, 0], t[:, 1]), 0.05) ** 2


def mlp_mse_grad(Ws, bs, x, target, row_weight=None):
    sizes = np.array([Ws[0].shape[1]] + [w.shape[0] for w in Ws], np.int32)
    Wc, bc, Wp, bp = _layer_ptrs(Ws, bs)
    gW = [np.zeros(w.shape, np.float64) for w in Ws]
    gb = [np.zeros(b.shape, np.float64) for b in bs]
    gWp = (C.c_void_p * len(gW))(*[_ptr(g) for g in gW])
    gbp = (C.c_void_p * len(gb))(*[_ptr(g) for g in gb])
    x = np.ascontiguousarray(x, np.float32)
    t = np.ascontiguousarray(target, np.float32)
    w = None if row_weight is None else np.ascontiguousarray(row_weight, np.float64)
    loss = lib().or_mlp_mse_grad(len(Ws), _ptr(sizes), Wp, bp, x.shape[0], _ptr(x), _ptr(t), _ptr(w), gWp, gbp)
    return loss, gW, gb


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam on float32 ``w`` with float64 moments ``m``, ``v``."""
    assert w.dtype == np.float32 and m.dtype == np.float64 and v.dtype == np.float64
    g = np.ascontiguousarray(g, np.float64)
    lib().or_adam(w.size, _ptr(w), _ptr(g), _ptr(m), _ptr(v), int(step), lr, b1, b2, eps)


def actor_critic(params, obs, counts):
    """Late-fusion actor-critic forward in FP64 (bf16 rounding points as set
    by set_bf16): mean [M, 3] and value [M]."""
    params = np.ascontiguousarray(params, np.float32)
    assert params.size == AC_PARAMS
    obs = np.ascontiguousarray(obs, np.float32).reshape(-1, FULL_DIM)
    counts = np.ascontiguousarray(counts, np.int32).reshape(-1, 2)
    M = obs.shape[0]
    mean = np.zeros((M, 3), np.float64)
    value = np.zeros(M, np.float64)
    lib().or_actor_critic(_ptr(params), M, _ptr(obs), _ptr(counts), _ptr(mean), _ptr(value))
    return mean, value
