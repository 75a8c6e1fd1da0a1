"""ctypes binding of ``libsf.so`` (the C ABI in ``include/sf.h``).

Argument marshalling only: every step of the simulation runs in the HIP
kernels behind the C ABI.  PyTorch provides device memory (tensors passed
as raw pointers) and the stream.  Loading fails loudly when the library has
not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SF_LIBRARY names another build of the same library (the AddressSanitizer
# build of the host code, for the CPU-side tests run under it)
LIB_PATH = os.environ.get("SF_LIBRARY") or os.path.join(HERE, "libsf.so")

SF_INVINCIBLE, SF_AUTO_RESET, SF_RECORD_CONTACTS = 1, 2, 4
NOALLOC_MAX_SAMPLES = 1 << 18      # SF_NOALLOC_MAX_SAMPLES of include/sf.h
FULL_EGO, FULL_ROAD_K, FULL_NEIGH_K = 11, 350, 24
FULL_DIM = FULL_EGO + 5 * FULL_ROAD_K + 7 * FULL_NEIGH_K
AC_BODY = (11 * 64 + 64 + 64 * 64 + 64 + 5 * 96 + 96 + 96 * 96 + 96 + 7 * 96 + 96 + 96 * 96 + 96
           + 256 * 128 + 128 + 128 * 64 + 64)
AC_PARAMS = 2 * AC_BODY + 3 * 64 + 3 + 3 + 64 + 1
EV_GOAL, EV_COLLISION, EV_CRASH, EV_TIMEOUT, EV_NUMERIC, EV_NAN_ACTION = 1, 2, 4, 8, 16, 32
EV_CONTACT_OVERFLOW = 64
EV_LANE_FORBIDDEN = 128
MAX_CONTACTS_PER_WORLD = 512
NF, NI, OBS_DIM = 24, 4, 256
FIELDS = ["px", "py", "pz", "qw", "qx", "qy", "qz", "vx", "vy", "vz", "wx", "wy", "wz",
          "om0", "om1", "om2", "om3", "steer", "steer_rate", "mu", "goal_x", "goal_y",
          "start_x", "start_y"]
IFIELDS = ["active", "ep_step", "since_spawn", "episode"]


class VehicleParams(C.Structure):
    _fields_ = [
        ("mass", C.c_float), ("inertia", C.c_float * 3),
        ("wheel_radius", C.c_float), ("wheel_mass", C.c_float), ("wheel_inertia", C.c_float),
        ("susp_k", C.c_float), ("susp_c", C.c_float), ("susp_rest", C.c_float),
        ("mount", (C.c_float * 3) * 4),
        ("length", C.c_float), ("width", C.c_float), ("wheelbase", C.c_float),
        ("tau_drive", C.c_float), ("tau_brake_front", C.c_float), ("tau_brake_rear", C.c_float),
        ("steer_kp", C.c_float), ("steer_kd", C.c_float), ("steer_tau_max", C.c_float),
        ("steer_inertia", C.c_float), ("steer_max", C.c_float),
        ("c_kappa", C.c_float), ("c_alpha", C.c_float), ("v_eps", C.c_float),
        ("trail", C.c_float), ("yaw_damping", C.c_float), ("gravity", C.c_float),
        ("jacobi_iters", C.c_int32), ("baumgarte", C.c_float), ("slop", C.c_float),
    ]


class WorldDesc(C.Structure):
    _fields_ = [
        ("num_worlds", C.c_int32),
        ("agent_offsets", C.c_void_p),
        ("road_offsets", C.c_void_p), ("road_xy", C.c_void_p), ("road_type", C.c_void_p),
        ("tri_offsets", C.c_void_p), ("tri_verts", C.c_void_p), ("tri_surface", C.c_void_p),
        ("num_surfaces", C.c_int32), ("mu_class", C.c_void_p),
        ("film_mm", C.c_void_p), ("pavement", C.c_void_p),
        ("spawn_offsets", C.c_void_p), ("spawn", C.c_void_p),
        ("seed", C.c_uint64),
        ("road_dir", C.c_void_p),
    ]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Options(C.Structure):
    _fields_ = [
        ("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", C.c_void_p),
        ("max_episode_steps", C.c_int32), ("collision_warmup", C.c_int32),
        ("flags", C.c_uint32), ("grid_cell", C.c_float),
        ("step_block", C.c_int32), ("obs_waves", C.c_int32), ("policy_rows", C.c_int32),
        ("tri_cell", C.c_float), ("step_grid", C.c_int32), ("reserved", C.c_int32 * 3),
    ]


SUR_INPUTS, SUR_PARAMS, SUR_SAMPLE = 16, 35587, 20
# piecewise-constant Adam learning rates (lr, steps) used to fit the tire
# network; 40k steps of 8192 samples take about 3 s on one MI355X
SUR_SCHEDULE = ((2e-3, 40000), (1e-3, 30000), (3e-4, 20000), (1e-4, 10000))


class SurTrainOpts(C.Structure):
    _fields_ = [
        ("steps", C.c_int32), ("batch", C.c_int32),
        ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
        ("seed", C.c_uint64), ("init_seed", C.c_uint64), ("set_envelope", C.c_int32),
    ]


class PPOOpts(C.Structure):
    _fields_ = [
        ("horizon", C.c_int32), ("epochs", C.c_int32), ("minibatches", C.c_int32),
        ("gamma", C.c_float), ("lam", C.c_float), ("clip", C.c_float), ("value_coef", C.c_float),
        ("entropy_coef", C.c_float), ("max_grad_norm", C.c_float), ("lr", C.c_float), ("kl_target", C.c_float),
        ("lr_min", C.c_float), ("lr_max", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
    ]


class PPOStats(C.Structure):
    _fields_ = [("lr", C.c_float), ("kl", C.c_float), ("surrogate", C.c_float), ("value_loss", C.c_float),
                ("entropy", C.c_float), ("clip_fraction", C.c_float), ("grad_norm", C.c_float),
                ("steps", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Tuning(C.Structure):
    _fields_ = [("step_block", C.c_int32), ("step_grid", C.c_int32), ("obs_waves", C.c_int32),
                ("policy_rows", C.c_int32), ("step_us", C.c_float), ("obs_us", C.c_float),
                ("policy_us", C.c_float), ("grid_cell", C.c_float), ("tri_cell", C.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SFError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libsf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SFError(f"{LIB_PATH} is missing: build it with paper_2605_08528_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, st = C.c_void_p, C.c_int32, C.c_int
        L.sf_default_params.argtypes = [C.POINTER(VehicleParams)]
        L.sf_default_options.argtypes = [C.POINTER(Options)]
        L.sf_create.argtypes = [C.POINTER(WorldDesc), C.POINTER(VehicleParams), C.POINTER(Options),
                                C.POINTER(vp)]
        L.sf_destroy.argtypes = [vp]
        L.sf_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.sf_step.argtypes = [vp, vp, C.c_float, i32]
        L.sf_observe.argtypes = [vp, vp, vp, vp, vp]
        L.sf_output_ptrs.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]
        L.sf_reset.argtypes = [vp, vp]
        L.sf_contact_overflows.argtypes = [vp, vp, i32]
        L.sf_road_touch.argtypes = [vp, i32]
        L.sf_road_touch_read.argtypes = [vp, vp, vp, C.POINTER(i32)]
        L.sf_set_dynamics.argtypes = [vp, i32]
        L.sf_set_shaping.argtypes = [vp, i32]
        L.sf_profile_calibrate.argtypes = [vp, i32, C.c_double]
        L.sf_observe_full.argtypes = [vp, vp, vp]
        L.sf_actor_critic_load.argtypes = [vp, vp, C.c_size_t]
        L.sf_actor_critic.argtypes = [vp, vp, vp, C.c_int64, vp, vp]
        L.sf_step_actor_critic.argtypes = [vp, C.c_float, i32]
        L.sf_actor_critic_read.argtypes = [vp, vp, vp, vp, vp, vp]
        L.sf_ppo_default_opts.argtypes = [C.POINTER(PPOOpts)]
        L.sf_ppo_init.argtypes = [vp, C.POINTER(PPOOpts)]
        L.sf_ppo_rollout.argtypes = [vp, C.c_float, i32, vp]
        L.sf_ppo_advantages.argtypes = [vp]
        L.sf_ppo_update.argtypes = [vp, vp, C.POINTER(PPOStats)]
        L.sf_ppo_gradient.argtypes = [vp, vp, i32, vp, vp]
        L.sf_ppo_read.argtypes = [vp] + [vp] * 10
        L.sf_actor_critic_get.argtypes = [vp, vp]
        L.sf_set_triangle_friction.argtypes = [vp, vp]
        L.sf_state_bytes.argtypes = [vp]
        L.sf_state_bytes.restype = C.c_size_t
        L.sf_get_state.argtypes = [vp, vp, C.c_size_t]
        L.sf_set_state.argtypes = [vp, vp, C.c_size_t]
        L.sf_get_contacts.argtypes = [vp, i32, vp, vp, i32]
        L.sf_debug_raycast.argtypes = [vp, vp]
        L.sf_debug_obs_indices.argtypes = [vp, vp]
        L.sf_policy_load.argtypes = [vp, vp, C.c_size_t]
        L.sf_policy_act.argtypes = [vp, vp]
        L.sf_step_policy.argtypes = [vp, C.c_float, i32]
        L.sf_graph_capture.argtypes = [vp, i32, C.c_float, i32]
        L.sf_graph_launch.argtypes = [vp]
        L.sf_profile.argtypes = [vp, i32]
        L.sf_profile_read.argtypes = [vp, vp, vp]
        L.sf_sur_log.argtypes = [vp, C.c_int64]
        L.sf_sur_collect.argtypes = [vp, vp, C.c_int64, C.POINTER(C.c_int64)]
        L.sf_sur_train.argtypes = [vp, vp, C.c_int64, C.POINTER(SurTrainOpts), C.POINTER(C.c_float)]
        L.sf_sur_gradient.argtypes = [vp, vp, C.c_int64, vp, C.POINTER(C.c_float)]
        L.sf_sur_predict.argtypes = [vp, vp, C.c_int64, vp]
        L.sf_sur_evaluate.argtypes = [vp, vp, C.c_int64, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.sf_sur_errors.argtypes = [vp, vp, C.c_int64, vp]
        L.sf_sur_errors_noalloc.argtypes = [vp, vp, C.c_int64, vp]
        L.sf_sur_set.argtypes = [vp, vp, vp, vp]
        L.sf_sur_get.argtypes = [vp, vp, vp, vp]
        L.sf_sur_enable.argtypes = [vp, i32]
        L.sf_sur_counts.argtypes = [vp, vp, i32]
        L.sf_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.sf_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.sf_autotune.argtypes = [vp, C.c_float, i32, i32, C.c_char_p, C.POINTER(Tuning)]
        L.sf_status_str.argtypes = [st]
        L.sf_status_str.restype = C.c_char_p
        L.sf_last_error.restype = C.c_char_p
        for name in ("sf_default_params", "sf_default_options", "sf_create", "sf_destroy", "sf_info",
                     "sf_step", "sf_observe", "sf_output_ptrs", "sf_reset", "sf_contact_overflows",
                     "sf_road_touch", "sf_road_touch_read", "sf_set_dynamics", "sf_set_shaping", "sf_ppo_default_opts", "sf_ppo_init", "sf_ppo_rollout",
                     "sf_ppo_advantages", "sf_ppo_update", "sf_ppo_gradient", "sf_ppo_read", "sf_actor_critic_get", "sf_profile_calibrate", "sf_set_triangle_friction",
                     "sf_observe_full", "sf_actor_critic_load", "sf_actor_critic", "sf_step_actor_critic",
                     "sf_actor_critic_read",
                     "sf_get_state",
                     "sf_set_state", "sf_get_contacts", "sf_debug_raycast", "sf_debug_obs_indices",
                     "sf_policy_load", "sf_policy_act", "sf_step_policy", "sf_graph_capture",
                     "sf_graph_launch", "sf_profile", "sf_profile_read", "sf_sur_log", "sf_sur_collect",
                     "sf_sur_train", "sf_sur_gradient", "sf_sur_predict", "sf_sur_evaluate", "sf_sur_errors",
                     "sf_sur_errors_noalloc", "sf_sur_set",
                     "sf_sur_get", "sf_sur_enable", "sf_sur_counts", "sf_get_tuning", "sf_set_tuning",
                     "sf_autotune"):
            getattr(L, name).restype = st
        _lib = L
    return _lib


def check(status: int, what: str = "") -> None:
    if status != 0:
        L = lib()
        raise SFError(f"{what}: {L.sf_status_str(status).decode()} ({L.sf_last_error().decode()})")


def make_params(prm: dict) -> VehicleParams:
    p = VehicleParams()
    for name, _ in VehicleParams._fields_:
        v = prm[name]
        if name == "inertia":
            for k in range(3):
                p.inertia[k] = v[k]
        elif name == "mount":
            for r in range(4):
                for c in range(3):
                    p.mount[r][c] = v[r][c]
        else:
            setattr(p, name, v)
    return p


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _tptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Sim:
    """One handle of W worlds on the current torch CUDA device."""

    def __init__(self, worlds, params: dict, flags: int = 0, stream=None, grid_cell: float = 0.0,
                 step_block: int = 0, obs_waves: int = 0, policy_rows: int = 0,
                 tri_cell: float = 0.0, step_grid: int = 0, torch_alloc: bool = True):
        import torch
        L = lib()
        self.torch = torch
        self.worlds = worlds
        self.params = dict(params)
        keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return _ptr(a)

        d = WorldDesc()
        d.num_worlds = worlds.num_worlds
        d.agent_offsets = arr(worlds.agent_offsets, np.int32)
        d.road_offsets = arr(worlds.road_offsets, np.int32)
        d.road_xy = arr(worlds.road_xy, np.float32)
        d.road_type = arr(worlds.road_type, np.uint8)
        d.tri_offsets = arr(worlds.tri_offsets, np.int32)
        d.tri_verts = arr(worlds.tri_verts, np.float32)
        d.tri_surface = arr(worlds.tri_surface, np.uint8)
        d.num_surfaces = worlds.num_surfaces
        d.mu_class = arr(worlds.mu_class, np.float32)
        d.film_mm = arr(worlds.film_mm, np.float32)
        d.pavement = arr(worlds.pavement, np.uint8)
        d.spawn_offsets = arr(worlds.spawn_offsets, np.int32)
        d.spawn = arr(worlds.spawn, np.float32)
        d.seed = int(worlds.seed)
        if getattr(worlds, "road_dir", None) is not None:
            d.road_dir = arr(worlds.road_dir, np.float32)
        o = Options()
        check(L.sf_default_options(C.byref(o)), "sf_default_options")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        o.stream = C.c_void_p(self.stream.cuda_stream)
        o.max_episode_steps = int(params.get("max_episode_steps", 1500))
        o.collision_warmup = int(params.get("collision_warmup", 24))
        o.flags = int(flags)
        o.grid_cell = float(grid_cell)
        o.step_block = int(step_block)
        o.obs_waves = int(obs_waves)
        o.policy_rows = int(policy_rows)
        o.tri_cell = float(tri_cell)
        o.step_grid = int(step_grid)
        # device memory from torch's caching allocator
        self._blocks = {}
        if torch_alloc:
            dev = torch.device("cuda", torch.cuda.current_device())

            def _alloc(nbytes, ctx):
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
                self._blocks[t.data_ptr()] = t
                return t.data_ptr()

            def _free(ptr, ctx):
                self._blocks.pop(ptr, None)

            self._alloc_cb = ALLOC_FN(_alloc)
            self._free_cb = FREE_FN(_free)
            o.alloc = self._alloc_cb
            o.free = self._free_cb
        h = C.c_void_p()
        check(L.sf_create(C.byref(d), C.byref(make_params(params)), C.byref(o), C.byref(h)), "sf_create")
        self.h = h
        W, N, A = C.c_int32(), C.c_int32(), C.c_int32()
        check(L.sf_info(h, C.byref(W), C.byref(N), C.byref(A)), "sf_info")
        self.W, self.N, self.max_agents = W.value, N.value, A.value
        self.flags = flags
        ob, rw, dn, ev = C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_void_p()
        check(L.sf_output_ptrs(h, C.byref(ob), C.byref(rw), C.byref(dn), C.byref(ev)), "sf_output_ptrs")
        self._out_ptrs = (ob.value, rw.value, dn.value, ev.value)

    def close(self):
        if getattr(self, "h", None):
            check(lib().sf_destroy(self.h), "sf_destroy")
            self.h = None
            self._blocks.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # calls ---------------------------------------------------------------
    def step(self, actions, dt: float, substeps: int) -> None:
        """actions: float32 CUDA tensor [N, 2] (a_long, steer)."""
        t = self.torch
        assert actions.is_cuda and actions.dtype == t.float32 and actions.is_contiguous()
        assert tuple(actions.shape) == (self.N, 2)
        check(lib().sf_step(self.h, _tptr(actions), C.c_float(dt), int(substeps)), "sf_step")

    def observe(self):
        """(obs [N,256] f32, reward [N] f32, done [N] u8, events [N] u8) CUDA tensors."""
        t = self.torch
        dev = t.device("cuda", t.cuda.current_device())
        obs = t.empty((self.N, OBS_DIM), dtype=t.float32, device=dev)
        rew = t.empty(self.N, dtype=t.float32, device=dev)
        done = t.empty(self.N, dtype=t.uint8, device=dev)
        ev = t.empty(self.N, dtype=t.uint8, device=dev)
        check(lib().sf_observe(self.h, _tptr(obs), _tptr(rew), _tptr(done), _tptr(ev)), "sf_observe")
        return obs, rew, done, ev

    def reset(self, mask) -> None:
        """mask: uint8 CUDA tensor [N]."""
        assert mask.is_cuda and mask.dtype == self.torch.uint8 and mask.numel() == self.N
        check(lib().sf_reset(self.h, _tptr(mask.contiguous())), "sf_reset")

    def contact_overflows(self, reset: bool = False) -> int:
        """(world, substep) solves that had more contact points than the
        per-world capacity since the counter was last cleared."""
        out = np.zeros(1, np.uint64)
        check(lib().sf_contact_overflows(self.h, _ptr(out), int(bool(reset))), "sf_contact_overflows")
        return int(out[0])

    def road_touch(self, enable: bool) -> None:
        """Count the distinct road items the step and observation kernels read
        in each following eager step (for the roofline's algorithmic bytes)."""
        check(lib().sf_road_touch(self.h, int(bool(enable))), "sf_road_touch")

    def road_touch_read(self):
        """(items [2, 6], bytes [2], steps): distinct road items read, summed over
        the counted steps, by the step kernel and the observation kernel."""
        items = np.zeros(12, np.uint64)
        nbytes = np.zeros(2, np.uint64)
        steps = C.c_int32()
        check(lib().sf_road_touch_read(self.h, _ptr(items), _ptr(nbytes), C.byref(steps)),
              "sf_road_touch_read")
        return items.reshape(2, 6).astype(np.int64), nbytes.astype(np.int64), steps.value

    # the paper's observation and network ---------------------------------
    def observe_full(self):
        """(obs [N, 1929], counts [N, 2]) CUDA tensors of the current state."""
        t = self.torch
        dev = t.device("cuda", t.cuda.current_device())
        obs = t.empty((self.N, FULL_DIM), dtype=t.float32, device=dev)
        cnt = t.empty((self.N, 2), dtype=t.int32, device=dev)
        check(lib().sf_observe_full(self.h, _tptr(obs), _tptr(cnt)), "sf_observe_full")
        return obs, cnt

    def actor_critic_load(self, params) -> None:
        a = np.ascontiguousarray(params, np.float32)
        assert a.size == AC_PARAMS
        check(lib().sf_actor_critic_load(self.h, _ptr(a), a.size), "sf_actor_critic_load")

    def actor_critic(self, obs, counts):
        """(mean [M, 3], value [M]) for CUDA rows obs [M, 1929], counts [M, 2]."""
        t = self.torch
        M = obs.shape[0]
        mean = t.empty((M, 3), dtype=t.float32, device=obs.device)
        value = t.empty(M, dtype=t.float32, device=obs.device)
        check(lib().sf_actor_critic(self.h, _tptr(obs.contiguous()), _tptr(counts.contiguous()), M, _tptr(mean),
                                    _tptr(value)), "sf_actor_critic")
        return mean, value

    def step_actor_critic(self, dt: float, substeps: int) -> None:
        check(lib().sf_step_actor_critic(self.h, float(dt), int(substeps)), "sf_step_actor_critic")

    def actor_critic_read(self):
        """Copies of the handle's last actor-critic outputs and observation:
        (mean [N, 3], value [N], actions [N, 2], obs [N, 1929], counts [N, 2])."""
        t = self.torch
        dev = t.device("cuda", t.cuda.current_device())
        mean = t.empty((self.N, 3), dtype=t.float32, device=dev)
        value = t.empty(self.N, dtype=t.float32, device=dev)
        act = t.empty((self.N, 2), dtype=t.float32, device=dev)
        obs = t.empty((self.N, FULL_DIM), dtype=t.float32, device=dev)
        cnt = t.empty((self.N, 2), dtype=t.int32, device=dev)
        check(lib().sf_actor_critic_read(self.h, _tptr(mean), _tptr(value), _tptr(act), _tptr(obs), _tptr(cnt)),
              "sf_actor_critic_read")
        return mean, value, act, obs, cnt

    def actor_critic_get(self):
        P = np.zeros(AC_PARAMS, np.float32)
        check(lib().sf_actor_critic_get(self.h, _ptr(P)), "sf_actor_critic_get")
        return P

    # on-device PPO -------------------------------------------------------
    @staticmethod
    def ppo_default_opts() -> dict:
        o = PPOOpts()
        check(lib().sf_ppo_default_opts(C.byref(o)), "sf_ppo_default_opts")
        return {k: getattr(o, k) for k, _ in PPOOpts._fields_}

    def ppo_init(self, **over) -> dict:
        d = self.ppo_default_opts()
        d.update(over)
        o = PPOOpts(**d)
        check(lib().sf_ppo_init(self.h, C.byref(o)), "sf_ppo_init")
        self.ppo_opts = d
        return d

    def ppo_rollout(self, eps, dt: float, substeps: int) -> None:
        """eps: CUDA float32 [T, N, 3] standard normals."""
        T = self.ppo_opts["horizon"]
        assert tuple(eps.shape) == (T, self.N, 3) and eps.dtype == self.torch.float32
        check(lib().sf_ppo_rollout(self.h, float(dt), int(substeps), _tptr(eps.contiguous())), "sf_ppo_rollout")

    def ppo_advantages(self) -> None:
        check(lib().sf_ppo_advantages(self.h), "sf_ppo_advantages")

    def ppo_update(self, perm) -> dict:
        """perm: CUDA int32 [epochs, N T], each row a permutation."""
        o = self.ppo_opts
        assert tuple(perm.shape) == (o["epochs"], o["horizon"] * self.N) and perm.dtype == self.torch.int32
        st = PPOStats()
        check(lib().sf_ppo_update(self.h, _tptr(perm.contiguous()), C.byref(st)), "sf_ppo_update")
        return st.as_dict()

    def ppo_gradient(self, rows):
        """(grad [AC_PARAMS] float32, stats [8] float64) on CUDA int32 rows."""
        g = np.zeros(AC_PARAMS, np.float32)
        st = np.zeros(8, np.float64)
        check(lib().sf_ppo_gradient(self.h, _tptr(rows.contiguous()), int(rows.numel()), _ptr(g), _ptr(st)),
              "sf_ppo_gradient")
        return g, st

    def ppo_read(self, advantages: bool = True) -> dict:
        """CUDA copies of the kept rollout."""
        t = self.torch
        dev = t.device("cuda", t.cuda.current_device())
        T, N = self.ppo_opts["horizon"], self.N
        f = lambda *shape: t.empty(shape, dtype=t.float32, device=dev)
        out = {"u": f(T, N, 3), "mean": f(T, N, 3), "logp": f(T, N), "value": f(T + 1, N), "reward": f(T, N),
               "done": t.empty((T, N), dtype=t.uint8, device=dev), "obs": f(T, N, FULL_DIM),
               "counts": t.empty((T, N, 2), dtype=t.int32, device=dev)}
        if advantages:
            out["adv"], out["ret"] = f(T, N), f(T, N)
        check(lib().sf_ppo_read(self.h, _tptr(out["u"]), _tptr(out["mean"]), _tptr(out["logp"]),
                                _tptr(out["value"]), _tptr(out["reward"]), _tptr(out["done"]),
                                _tptr(out["adv"]) if advantages else None, _tptr(out["ret"]) if advantages else None,
                                _tptr(out["obs"]), _tptr(out["counts"])), "sf_ppo_read")
        return out

    def set_dynamics(self, mode: str) -> None:
        """'physics' (the articulated vehicle) or 'bicycle' (kinematic model)."""
        check(lib().sf_set_dynamics(self.h, {"physics": 0, "bicycle": 1}[mode]), "sf_set_dynamics")

    def set_shaping(self, on: bool) -> None:
        """Dense shaping rewards and the lane-forbidden termination on or off."""
        check(lib().sf_set_shaping(self.h, 1 if on else 0), "sf_set_shaping")

    def set_triangle_friction(self, scale) -> None:
        """Friction factor per road triangle [T] (None: back to 1)."""
        if scale is None:
            check(lib().sf_set_triangle_friction(self.h, None), "sf_set_triangle_friction")
            return
        a = np.ascontiguousarray(scale, np.float32)
        assert a.size == len(self.worlds.tri_surface)
        check(lib().sf_set_triangle_friction(self.h, _ptr(a)), "sf_set_triangle_friction")

    def state_bytes(self) -> int:
        return int(lib().sf_state_bytes(self.h))

    def get_state(self):
        """(f [24, N] float32, k [4, N] int32) host copies."""
        buf = np.zeros(self.state_bytes() // 4, np.float32)
        check(lib().sf_get_state(self.h, _ptr(buf), buf.nbytes), "sf_get_state")
        f = buf[:NF * self.N].reshape(NF, self.N).copy()
        k = buf[NF * self.N:].view(np.int32).reshape(NI, self.N).copy()
        return f, k

    def set_state(self, f, k) -> None:
        f = np.ascontiguousarray(f, np.float32).reshape(NF, self.N)
        k = np.ascontiguousarray(k, np.int32).reshape(NI, self.N)
        buf = np.concatenate([f.ravel(), k.ravel().view(np.float32)])
        check(lib().sf_set_state(self.h, _ptr(buf), buf.nbytes), "sf_set_state")

    def contacts(self, substep: int):
        """(counts [W] int32, pairs [W, cap] uint32) of one substep of the last step."""
        cap = max(1, self.max_agents * (self.max_agents - 1) // 2)
        cnt = np.zeros(self.W, np.int32)
        pairs = np.zeros((self.W, cap), np.uint32)
        check(lib().sf_get_contacts(self.h, int(substep), _ptr(cnt), _ptr(pairs), cap), "sf_get_contacts")
        return cnt, pairs

    def debug_raycast(self):
        out = np.zeros((self.N, 4, 4), np.float32)
        check(lib().sf_debug_raycast(self.h, _ptr(out)), "sf_debug_raycast")
        return out

    def debug_obs_indices(self):
        out = np.zeros((self.N, 72), np.int32)
        check(lib().sf_debug_obs_indices(self.h, _ptr(out)), "sf_debug_obs_indices")
        return out

    # policy, graphs, profiling ------------------------------------------
    def policy_load(self, Ws, bs) -> None:
        """Float32 masters of the 256-256-256-2 policy (W as [out, in])."""
        flat = np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(),
                                               np.asarray(b, np.float32).ravel()])
                               for W, b in zip(Ws, bs)])
        check(lib().sf_policy_load(self.h, _ptr(flat), flat.size), "sf_policy_load")

    def policy_act(self):
        t = self.torch
        a = t.empty((self.N, 2), dtype=t.float32, device=t.device("cuda", t.cuda.current_device()))
        check(lib().sf_policy_act(self.h, _tptr(a)), "sf_policy_act")
        return a

    def step_policy(self, dt: float, substeps: int) -> None:
        check(lib().sf_step_policy(self.h, C.c_float(dt), int(substeps)), "sf_step_policy")

    def graph_capture(self, control_steps: int, dt: float, substeps: int) -> None:
        check(lib().sf_graph_capture(self.h, int(control_steps), C.c_float(dt), int(substeps)),
              "sf_graph_capture")

    def graph_launch(self) -> None:
        check(lib().sf_graph_launch(self.h), "sf_graph_launch")

    def profile(self, enable: bool) -> None:
        check(lib().sf_profile(self.h, int(bool(enable))), "sf_profile")

    def profile_read(self):
        """{kernel: (total_ms, launches)} for policy, step, obs, reset, the
        paper-shaped observation, the actor-critic, the clock kernels and the PPO
        backward pass."""
        ms = np.zeros(8, np.float64)
        n = np.zeros(8, np.int32)
        check(lib().sf_profile_read(self.h, _ptr(ms), _ptr(n)), "sf_profile_read")
        return {k: (float(ms[i]), int(n[i]))
                for i, k in enumerate(("policy", "step", "obs", "reset", "obs_full", "actor_critic", "clock",
                                       "ppo_backward"))}

    def profile_calibrate(self, n: int = 20, us: float = 50.0) -> None:
        """n wall-clock kernels of `us` microseconds timed like the others."""
        check(lib().sf_profile_calibrate(self.h, int(n), float(us)), "sf_profile_calibrate")

    # learned tire surrogate --------------------------------------------
    def sur_log(self, capacity: int) -> None:
        check(lib().sf_sur_log(self.h, int(capacity)), "sf_sur_log")

    def sur_collect(self, max_out: int):
        """Valid logged samples as a [n, 20] device tensor (n <= max_out)."""
        t = self.torch
        out = t.empty((max(int(max_out), 1), SUR_SAMPLE), dtype=t.float32,
                      device=t.device("cuda", t.cuda.current_device()))
        n = C.c_int64()
        check(lib().sf_sur_collect(self.h, _tptr(out), int(max_out), C.byref(n)), "sf_sur_collect")
        return out[:min(n.value, int(max_out))], n.value

    def sur_train(self, data, steps: int, batch: int = 4096, lr: float = 1e-3, beta1: float = 0.9,
                  beta2: float = 0.999, eps: float = 1e-8, seed: int = 1, init_seed: int = 0,
                  set_envelope: bool = False) -> float:
        o = SurTrainOpts(int(steps), int(batch), lr, beta1, beta2, eps, int(seed), int(init_seed),
                         int(bool(set_envelope)))
        loss = C.c_float()
        check(lib().sf_sur_train(self.h, _tptr(data), data.shape[0], C.byref(o), C.byref(loss)),
              "sf_sur_train")
        return loss.value

    def sur_fit(self, data, schedule=SUR_SCHEDULE, batch: int = 8192, init_seed: int = 1) -> float:
        """Fresh network and envelope from ``data``, then the Adam phases of
        ``schedule``; returns the last minibatch loss."""
        self.sur_train(data, steps=0, init_seed=init_seed, set_envelope=True)
        loss = float("nan")
        for k, (lr, n) in enumerate(schedule):
            loss = self.sur_train(data, steps=n, batch=batch, lr=lr, seed=k + 1)
        return loss

    def sur_gradient(self, data):
        g = np.zeros(SUR_PARAMS, np.float32)
        loss = C.c_float()
        check(lib().sf_sur_gradient(self.h, _tptr(data), data.shape[0], _ptr(g), C.byref(loss)),
              "sf_sur_gradient")
        return loss.value, g

    def sur_predict(self, data):
        t = self.torch
        out = t.empty((data.shape[0], 3), dtype=t.float32, device=data.device)
        check(lib().sf_sur_predict(self.h, _tptr(data), data.shape[0], _tptr(out)), "sf_sur_predict")
        return out

    def sur_evaluate(self, data):
        m, p = C.c_float(), C.c_float()
        check(lib().sf_sur_evaluate(self.h, _tptr(data), data.shape[0], C.byref(m), C.byref(p)),
              "sf_sur_evaluate")
        return m.value, p.value

    def sur_errors(self, data):
        """Per-sample relative force error of the network on data [M][20] (CUDA tensor [M])."""
        t = self.torch
        e = t.empty(data.shape[0], dtype=t.float32, device=data.device)
        check(lib().sf_sur_errors(self.h, _tptr(data), data.shape[0], _tptr(e)), "sf_sur_errors")
        return e

    def sur_errors_noalloc(self, data, out):
        """The same errors written into a caller-provided CUDA tensor out [M];
        the library allocates nothing (its predictions use a fixed per-GPU
        scratch of at most NOALLOC_MAX_SAMPLES samples)."""
        assert out.is_cuda and out.dtype == self.torch.float32 and out.numel() >= data.shape[0]
        check(lib().sf_sur_errors_noalloc(self.h, _tptr(data), data.shape[0], _tptr(out)),
              "sf_sur_errors_noalloc")
        return out

    def sur_set(self, params, lo, hi) -> None:
        self._sur_keep = [np.ascontiguousarray(a, np.float32) for a in (params, lo, hi)]
        check(lib().sf_sur_set(self.h, *[_ptr(a) for a in self._sur_keep]), "sf_sur_set")

    def sur_get(self):
        p = np.zeros(SUR_PARAMS, np.float32)
        lo = np.zeros(SUR_INPUTS, np.float32)
        hi = np.zeros(SUR_INPUTS, np.float32)
        check(lib().sf_sur_get(self.h, _ptr(p), _ptr(lo), _ptr(hi)), "sf_sur_get")
        return p, lo, hi

    def sur_enable(self, on: bool) -> None:
        check(lib().sf_sur_enable(self.h, int(bool(on))), "sf_sur_enable")

    def sur_counts(self, reset: bool = False):
        out = np.zeros(2, np.uint64)
        check(lib().sf_sur_counts(self.h, _ptr(out), int(bool(reset))), "sf_sur_counts")
        return int(out[0]), int(out[1])

    # launch shapes ------------------------------------------------------
    def tuning(self) -> dict:
        t = Tuning()
        check(lib().sf_get_tuning(self.h, C.byref(t)), "sf_get_tuning")
        return t.as_dict()

    def set_tuning(self, step_block: int, step_grid: int, obs_waves: int, policy_rows: int,
                   grid_cell: float = 0.0, tri_cell: float = 0.0) -> None:
        """Launch shapes; cell sizes of 0 keep the current grids, others rebuild them."""
        t = Tuning(int(step_block), int(step_grid), int(obs_waves), int(policy_rows), 0.0, 0.0, 0.0,
                   float(grid_cell), float(tri_cell))
        check(lib().sf_set_tuning(self.h, C.byref(t)), "sf_set_tuning")

    def autotune(self, dt: float, substeps: int, steps: int = 20, cache_path: str | None = None) -> dict:
        t = Tuning()
        path = cache_path.encode() if cache_path else None
        check(lib().sf_autotune(self.h, C.c_float(dt), int(substeps), int(steps), path, C.byref(t)),
              "sf_autotune")
        return t.as_dict()
