#!/usr/bin/env python3
"""Throughput of the batched driving-physics control step on one MI355X.

A step is one pass of the whole hot path over the workload: policy MLP on
the current observations, the fused physics step (4 substeps of steering,
raycast suspension, tire and spin, chassis, vehicle-vehicle contact,
integration, events, rewards, in-step respawn) and the observation gather
(which, in the autotuner's usual pick, also evaluates the policy for the
next step).  The default workload is 256 worlds with 4-32 vehicles each
(4096 in total) on procedural road grids of 1k-20k points, dt = 1/30 s with
4 substeps.

Prints one JSON line: controlled-agent steps per second (CASPS) over the
timed steps, run as replays of captured graphs of up to 16 control steps and
averaged over three seeded workloads; the dominant kernel against its
roofline (per-kernel HIP events on the stream the kernels run on, from a
profiled eager pass over the same number of steps); and the FP64 CPU
oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "controlled-agent steps/s @256 worlds×16 agents; plain vs surrogate step"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
# Algorithmic bytes per controlled agent and control step (the state stays
# in registers/LDS across substeps): the step kernel reads the state (76 B
# dynamic + 8 B counters + 16 B start and goal) and the actions (8 B) and
# writes the state (76 + 8 B) and reward, done and events (6 B); the
# observation kernel writes the 1 KB observation row.  Road bytes come on
# top: the distinct grid ranges, triangle records and road points each
# kernel reads, counted in the kernels during a separate eager pass.
STEP_BYTES_PER_AGENT = (76 + 8 + 16) + (76 + 8) + 8 + 6
OBS_BYTES_PER_AGENT = 1024
CONTROL_STEP_BYTES_PER_AGENT = STEP_BYTES_PER_AGENT + OBS_BYTES_PER_AGENT
POLICY_FLOP_PER_AGENT = 2 * (256 * 256 * 2 + 256 * 2)
POLICY_WEIGHT_BYTES = 132098 * 2              # bf16 copies of the three layers read once per launch
TOUCH_STEPS = 20                              # eager steps of the road-touch counting pass
SETTLE_STEPS = 300                            # control steps from spawn to the measured traffic state
# learned tire network 16 -> 128 -> 128 -> 128 -> 3: multiply-adds per evaluation,
# and forward + backward (weight and input gradients) per training sample
SUR_FLOP_PER_EVAL = 2 * (16 * 128 + 128 * 128 * 2 + 128 * 3)
SUR_TRAIN_FLOP_PER_SAMPLE = 3 * SUR_FLOP_PER_EVAL
ACT_BYTES_PER_AGENT = 8                       # two float actions written


def obs_bytes(n_agents: int, fused: bool, road: float = 0.0) -> float:
    """Algorithmic bytes of one observation launch: the rows written and the
    road data read; the kernel that also evaluates the policy reads the
    network once and writes the actions (the step reads them back)."""
    b = OBS_BYTES_PER_AGENT * n_agents + road
    return b + (POLICY_WEIGHT_BYTES + ACT_BYTES_PER_AGENT * n_agents if fused else 0)


def step_bytes(n_agents: int, road: float = 0.0) -> float:
    """Algorithmic bytes of one step launch (state, actions, outputs, road)."""
    return STEP_BYTES_PER_AGENT * n_agents + road


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def recorded_traffic(kernel: str, launch_name: str, n_agents: int):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    record (scaled by the copy-kernel calibration), or None when the kernel
    source changed since the counters were taken, or the launch shape or the
    workload size differs."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    k = rec.get("launches", {}).get(launch_name)
    from paper_2605_08528_amd.profile_summary import kernel_source_hash
    if not k or k.get("kernel") != kernel or k.get("source_hash") != kernel_source_hash(kernel) \
            or k.get("agents") != n_agents:
        return None
    return (k["fetch_kib"] * rec["fetch_scale"] + k["write_kib"] * rec["write_scale"]) * 1024.0


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(worlds, prm, dt, S, policy, seconds, max_worlds=16):
    """The FP64 oracle on the first worlds of the workload: observe -> policy
    -> step, timed over >= 20 control steps after 2 warm-up steps, first on
    one thread, then with OpenMP over worlds on every host thread (half of
    the time budget each)."""
    from oracle import oracle as O
    sub = worlds.world_slice(0, min(max_worlds, worlds.num_worlds))
    Ws, bs = policy

    def rate(threads, budget):
        orc = O.Oracle(sub, prm, auto_reset=True, threads=threads)

        def one():
            obs = orc.observe()
            act = O.policy(Ws, bs, obs, steer_max=prm["steer_max"]).astype(np.float32)
            orc.step(act, dt, S)

        for _ in range(2):
            one()
        t0 = time.perf_counter()
        n = 0
        while n < 20 or time.perf_counter() - t0 < budget:
            one()
            n += 1
            if time.perf_counter() - t0 > 3 * budget:
                break
        el = time.perf_counter() - t0
        return orc.N * n / el, n, orc.N

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    one_t, n1, N = rate(1, 0.5 * seconds)
    all_t, n, N = rate(threads, 0.5 * seconds)
    return {"value": all_t, "unit": "controlled-agent steps/s", "cores": threads,
            "kind": "oracle", "cpu": cpu_model(),
            "single_thread": {"value": one_t, "cores": 1, "steps": n1},
            "sample": f"first {sub.num_worlds} worlds ({N} agents) of the same workload, "
                      f"{n} control steps (observe, policy, step) on {threads} threads, "
                      f"{n1} on one thread; FP64 brute force"}


def _heading(f):
    hx = 1 - 2 * (f[5] ** 2 + f[6] ** 2)
    hy = 2 * (f[4] * f[5] + f[3] * f[6])
    L = np.maximum(np.hypot(hx, hy), 1e-6)
    return hx / L, hy / L


def trajectory_error(sim, torch, sf, dt, S, steps, v0=None, driving=False):
    """Position difference between the plain and the network step after
    `steps` control steps from the same state, over agents that neither
    run reset.  Optionally every vehicle first moves along its heading at
    v0 m/s; actions are the seeded random ones, or with `driving` a steady
    throttle of 0.35 and a slow steering sine (3 s period)."""
    from paper_2605_08528_amd import inputs as I
    f0, k0 = sim.get_state()
    if v0 is not None:
        hx, hy = _heading(f0)
        f0[7], f0[8] = v0 * hx, v0 * hy
        f0[13:17] = v0 / 0.35
    if driving:
        acts = []
        for t in range(steps):
            a = np.empty((sim.N, 2), np.float32)
            a[:, 0] = 0.35
            a[:, 1] = 0.1 * np.sin(2.0 * np.pi * t * dt / 3.0)
            acts.append(torch.from_numpy(a).cuda())
    else:
        acts = [torch.from_numpy(I.actions(7, t, sim.N)).cuda() for t in range(steps)]
    ends = []
    for on in (False, True):
        sim.set_state(f0, k0)
        sim.sur_enable(on)
        for a in acts:
            sim.step(a, dt, S)
        torch.cuda.synchronize()
        ends.append(sim.get_state())
    sim.sur_enable(False)
    (fa, ka), (fb, kb) = ends
    same = (ka[3] == k0[3]) & (kb[3] == k0[3]) & (k0[0] == 1)   # same episode, active at the start
    d = np.hypot(fa[0] - fb[0], fa[1] - fb[1])[same]
    moved = np.hypot(fa[0] - f0[0], fa[1] - f0[1])[same]
    return {"agents": int(same.sum()), "of": int(sim.N), "mean_m": float(d.mean()),
            "p95_m": float(np.percentile(d, 95)), "max_m": float(d.max()), "mean_path_m": float(moved.mean()),
            "actions": "throttle 0.35, steering 0.1 sin(2 pi t / 3 s)" if driving else "seeded uniform random",
            "initial_speed": v0}


def log_tire_samples(torch, sf, I, worlds, steps, seed, reinit=40, dt=1.0 / 30.0, S=4):
    """Samples of the plain tire model (inputs and outputs of every loaded
    wheel at |v_x| >= 3 m/s) from `steps` control steps of seeded random
    actions on `worlds`; every `reinit` steps every vehicle is launched
    again along its heading at U[3, 30] m/s with its wheels rolling."""
    sim = sf.Sim(worlds, dict(I.VEHICLE_DEFAULTS), flags=sf.SF_INVINCIBLE | sf.SF_AUTO_RESET)
    N = sim.N
    cap = steps * S * 4 * N
    sim.sur_log(cap)
    for t in range(steps):
        if t % reinit == 0:
            f, k = sim.get_state()
            spd = I.speeds(seed, t, N)
            hx, hy = _heading(f)
            f[7], f[8] = spd * hx, spd * hy
            f[13:17] = spd / 0.35
            sim.set_state(f, k)
        sim.step(torch.from_numpy(I.actions(seed, t, N)).cuda(), dt, S)
    data, n = sim.sur_collect(cap)
    sim.sur_log(0)
    torch.cuda.synchronize()
    sim.close()
    return data


def force_errors(sim, data):
    """Relative force error statistics of the current network on `data`."""
    e = sim.sur_errors(data).cpu().numpy().astype(np.float64)
    y = sim.sur_predict(data).cpu().numpy().astype(np.float64)
    t = data[:, 16:18].cpu().numpy().astype(np.float64)
    F = np.hypot(t[:, 0], t[:, 1])
    dF = np.hypot(y[:, 0] - t[:, 0], y[:, 1] - t[:, 1])
    return {"mean": float(e.mean()), "p50": float(np.percentile(e, 50)), "p95": float(np.percentile(e, 95)),
            "p99": float(np.percentile(e, 99)), "max": float(e.max()),
            "aggregate": float(dF.sum() / max(F.sum(), 1e-30)), "samples": int(len(e))}


def surrogate_leg(sim, torch, sf, I, stream, dt, S, steps, warmup, train_samples, main_log_steps):
    """The learned tire model: trained on samples of the plain step logged
    from the tire-sampling workload (1024 worlds x 16 agents, friction
    classes down to 0.001, random actions, launches at 3-30 m/s), judged on
    1 M samples of another run of it and on samples of the benchmark's own
    policy-driven workload; then the same control step with the network
    inside (wheels outside its envelope or failing the residual checks fall
    back to the plain tire model), timed like the plain step."""
    N = sim.N
    t0 = time.perf_counter()
    train = log_tire_samples(torch, sf, I, I.tire_sampling(seed=101), 80, 101)[:train_samples]
    held = log_tire_samples(torch, sf, I, I.tire_sampling(seed=202), 10, 202)[:1_000_000]
    cap = main_log_steps * S * 4 * N
    sim.sur_log(cap)
    for _ in range(main_log_steps):
        sim.step_policy(dt, S)
    held_main, _ = sim.sur_collect(cap)
    sim.sur_log(0)
    torch.cuda.synchronize()
    t_log = time.perf_counter() - t0
    sim.sur_train(train, steps=0, init_seed=1, set_envelope=True)
    untrained = force_errors(sim, held)
    t0 = time.perf_counter()
    loss = sim.sur_fit(train)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_adam = sum(k for _, k in sf.SUR_SCHEDULE)
    err = force_errors(sim, held)
    err_main = force_errors(sim, held_main)
    log(f"surrogate: {train.shape[0]} training samples ({t_log:.1f} s of logging), {n_adam} Adam steps in "
        f"{t_train:.1f} s; held-out force error mean {err['mean']:.4f} p99 {err['p99']:.4f}; on the "
        f"benchmark workload mean {err_main['mean']:.4f} (untrained {untrained['mean']:.3f})")
    n_train = int(train.shape[0])
    del train, held, held_main
    sim.sur_enable(True)
    for _ in range(warmup):
        sim.step_policy(dt, S)
    # the plain step's kernel over the same control steps from the same
    # state, so that the two kernels are compared on one load
    f0, k0 = sim.get_state()
    sim.sur_enable(False)
    sim.profile(True)
    for _ in range(steps):
        sim.step_policy(dt, S)
    torch.cuda.synchronize()
    ev_p, fixed_p = read_profile(sim)
    plain_us = kernel_us(ev_p, fixed_p)["step"]
    sim.set_state(f0, k0)
    sim.sur_enable(True)
    # profiled eager pass (per-kernel events, wheel counts), then the timed
    # region measured as the plain step is: replays of a captured graph
    sim.sur_counts(reset=True)
    sim.profile(True)
    for _ in range(steps):
        sim.step_policy(dt, S)
    torch.cuda.synchronize()
    ev, fixed = read_profile(sim)
    used, fb = sim.sur_counts(reset=True)
    G = graph_len(steps)
    sim.graph_capture(G, dt, S)
    sim.graph_launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps // G):
        sim.graph_launch()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sim.sur_enable(False)     # drops the graph
    casps = N * steps / (ms / 1e3)
    step_us = kernel_us(ev, fixed)["step"]
    # the network runs on every in-domain wheel-substep (fallback decided after)
    net_tflops = (used + fb) * SUR_FLOP_PER_EVAL / (steps * step_us * 1e-6) / 1e12
    train_tflops = n_adam * 8192 * SUR_TRAIN_FLOP_PER_SAMPLE / t_train / 1e12
    traj = trajectory_error(sim, torch, sf, dt, S, 200)
    log(f"surrogate step: {ms / steps:.4f} ms/step, {casps:.4g} CASPS, network on "
        f"{used / max(1, used + fb):.3f} of in-domain wheel-substeps")
    return {
        "value": casps, "unit": "controlled-agent steps/s", "ms_per_step": ms / steps,
        "timed": f"{steps} control steps as replays of {G}-step hipGraphs (profiling off), seed of the main leg",
        "step_kernel_us": step_us,
        "plain_step_kernel_us_same_steps": plain_us,
        "step_kernel_ratio": step_us / plain_us,
        "network_tflops_in_step": net_tflops, "train_tflops": train_tflops,
        "network_share": used / max(1, used + fb), "wheel_substeps_in_domain": used + fb,
        "force_error_heldout": err, "force_error_benchmark_workload": err_main,
        "force_error_untrained": untrained["mean"],
        "fallback_rate": fb / max(1, used + fb), "train_samples": n_train,
        "adam_steps": n_adam, "batch": 8192, "train_seconds": t_train, "last_loss": loss,
        "trajectory_error_200": traj,
        "note": "force error = |d(Fx,Fy)| / max(|(Fx,Fy)|, 0.05 mu Fz) per sample against the plain tire "
                "model; aggregate = sum |d(Fx,Fy)| / sum |(Fx,Fy)|; training: samples of 80 control steps "
                "of the tire-sampling workload (seed 101), held out: 1 M samples of another run (seed 202)",
    }


def config_leg(name, torch, sf, I, stream, steps, sur_params, tune_steps):
    """Context for the other workload sizes: graph-replay CASPS of the plain
    control step, per-kernel durations from a profiled eager pass, and the
    step with the learned tire model trained in the main leg (wheels outside
    its training envelope fall back to the plain model)."""
    w = I.workload(name)
    dt, S = I.TIMING[name]
    with torch.cuda.stream(stream):
        sim = sf.Sim(w, dict(I.VEHICLE_DEFAULTS), flags=sf.SF_AUTO_RESET, stream=stream)
        sim.policy_load(*I.mlp_params([256, 256, 256, 2], seed=0))
        N = sim.N
        for _ in range(100):
            sim.step_policy(dt, S)
        tuning = sim.autotune(dt, S, steps=tune_steps)
        sim.profile(True)
        for _ in range(steps):
            sim.step_policy(dt, S)
        torch.cuda.synchronize()
        ev, fixed = read_profile(sim)
        G = graph_len(steps)
        sim.graph_capture(G, dt, S)
        sim.graph_launch()
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record(stream)
        for _ in range(steps // G):
            sim.graph_launch()
        g1.record(stream)
        torch.cuda.synchronize()
        ms = g0.elapsed_time(g1)
        out = {"worlds": w.num_worlds, "agents": N, "steps": steps, "casps": N * steps / (ms / 1e3),
               "ms_per_step": ms / steps,
               "launch_shapes": {k: tuning[k] for k in ("step_block", "step_grid", "obs_waves", "policy_rows",
                                                          "grid_cell", "tri_cell")},
               "kernels_us": kernel_us(ev, fixed), "event_fixed_us": fixed}
        if "step" in out["kernels_us"]:
            out["step_algorithmic_gbs"] = step_bytes(N) / (out["kernels_us"]["step"] * 1e-6) / 1e9
        if sur_params is not None:
            # the same control step with the network inside, timed the same way
            sim.sur_set(*sur_params)
            sim.sur_enable(True)
            for _ in range(20):
                sim.step_policy(dt, S)
            sim.sur_counts(reset=True)
            sim.graph_capture(G, dt, S)
            sim.graph_launch()
            torch.cuda.synchronize()
            g0.record(stream)
            for _ in range(steps // G):
                sim.graph_launch()
            g1.record(stream)
            torch.cuda.synchronize()
            ms_s = g0.elapsed_time(g1)
            used, fb = sim.sur_counts(reset=True)
            sim.sur_enable(False)
            out["surrogate"] = {"casps": N * steps / (ms_s / 1e3), "ms_per_step": ms_s / steps,
                                "network_share": used / max(1, used + fb)}
            if name == "dense4096x32":
                # 200 control steps of driving from 10 m/s: plain against network
                out["surrogate"]["trajectory_error_200"] = trajectory_error(sim, torch, sf, dt, S, 200, v0=10.0,
                                                                            driving=True)
        sim.close()
    log(f"{name}: {N} agents, graph {out['ms_per_step']:.4f} ms/step, {out['casps']:.4g} CASPS"
        + (f"; surrogate {out['surrogate']['casps']:.4g} CASPS" if "surrogate" in out else ""))
    return out


def ac_flop(counts: np.ndarray) -> float:
    """Algorithmic FLOP of the late-fusion actor-critic on rows with these
    valid (road, neighbour) counts: both networks, every layer, no padding."""
    nr = counts[:, 0].astype(np.float64)
    nv = counts[:, 1].astype(np.float64)
    per_net = (11 * 64 + 64 * 64 + nr * (5 * 96 + 96 * 96) + nv * (7 * 96 + 96 * 96) + 256 * 128 + 128 * 64)
    return float(2.0 * (2 * per_net.sum() + len(nr) * 64 * (3 + 1)))


def ppo_leg(torch, sf, I, stream, workload, horizon, iters, seed=0):
    """On-device PPO with the paper's hyperparameters (horizon, 5 epochs x 16
    minibatches, dense shaping rewards on): `iters` iterations after one
    untimed, each a rollout of `horizon` control steps and the update, timed
    with HIP events; training CASPS = agents x horizon / iteration time, the
    quantity the paper's throughput is (it measures during PPO training).
    Per-kernel durations from a profiled iteration."""
    w = I.workload(workload, seed=seed)
    dt, S = I.TIMING[workload]
    with torch.cuda.stream(stream):
        sim = sf.Sim(w, dict(I.VEHICLE_DEFAULTS), flags=sf.SF_AUTO_RESET, stream=stream)
        rng = np.random.default_rng(seed)
        P = (rng.standard_normal(sf.AC_PARAMS) * 0.1).astype(np.float32)
        sim.actor_critic_load(P)
        sim.set_shaping(True)
        opts = sim.ppo_init(horizon=horizon)
        N, TN = sim.N, horizon * sim.N
        g = torch.Generator(device="cuda").manual_seed(seed)

        def iteration():
            eps = torch.randn((horizon, N, 3), generator=g, device="cuda", dtype=torch.float32)
            perm = torch.stack([torch.randperm(TN, generator=g, device="cuda") for _ in range(opts["epochs"])])
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record(stream)
            sim.ppo_rollout(eps, dt, S)
            e1.record(stream)
            st = sim.ppo_update(perm.to(torch.int32))
            e2.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1), e1.elapsed_time(e2), st

        iteration()                                   # untimed
        sim.profile(True)
        iteration()
        torch.cuda.synchronize()
        ev, fixed = read_profile(sim)
        times = [iteration() for _ in range(iters)]
        sim.close()
    roll = float(np.mean([t[0] for t in times]))
    upd = float(np.mean([t[1] for t in times]))
    us = kernel_us(ev, fixed)
    last = times[-1][2]
    return {"workload": workload, "agents": N, "horizon": horizon, "epochs": opts["epochs"],
            "minibatches": opts["minibatches"], "rows_per_minibatch": TN // opts["minibatches"],
            "iterations_timed": iters, "rollout_ms": roll, "update_ms": upd,
            "training_casps": TN / ((roll + upd) * 1e-3), "rollout_casps": TN / (roll * 1e-3),
            "kernels_us": us,
            "per_minibatch_us": {"forward_with_save": us.get("actor_critic", 0.0),
                                 "backward": us.get("ppo_backward", 0.0)},
            "last_update": last,
            "note": "rollout: observation, actor-critic, sampling, physics step per control step (eager); update: "
                    "advantages, then per minibatch the forward pass with saved activations, loss, backward, "
                    "reduction, clip and Adam; one host synchronisation per minibatch (the KL-adaptive rate); "
                    "actor_critic in kernels_us mixes rollout (4096 rows) and update (32768 rows) launches"}


def full_obs_leg(torch, sf, I, stream, workload, steps, seed=0):
    """The paper-shaped observation (1929 floats per agent) and the
    late-fusion actor-critic (seeded random weights) driving the physics
    step: control steps timed with HIP events around the whole sequence
    (eager launches), per-kernel durations from a profiled pass, the
    network's rate in algorithmic FLOP against the bf16 matrix-core peak and
    the observation's in algorithmic bytes against the HBM peak."""
    w = I.workload(workload, seed=seed)
    dt, S = I.TIMING[workload]
    with torch.cuda.stream(stream):
        sim = sf.Sim(w, dict(I.VEHICLE_DEFAULTS), flags=sf.SF_AUTO_RESET, stream=stream)
        rng = np.random.default_rng(seed)
        sim.actor_critic_load((rng.standard_normal(sf.AC_PARAMS) * 0.1).astype(np.float32))
        N = sim.N
        for _ in range(20):
            sim.step_actor_critic(dt, S)
        sim.profile(True)
        for _ in range(steps):
            sim.step_actor_critic(dt, S)
        torch.cuda.synchronize()
        ev, fixed = read_profile(sim)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            sim.step_actor_critic(dt, S)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        _, cnt = sim.observe_full()
        torch.cuda.synchronize()
        counts = cnt.cpu().numpy()
        sim.close()
    us = kernel_us(ev, fixed)
    flop = ac_flop(counts)
    obs_bytes_ = N * (sf.FULL_DIM * 4 + 8)
    out = {"workload": workload, "agents": N, "steps": steps, "casps_eager": N * steps / (ms / 1e3),
           "ms_per_step": ms / steps, "kernels_us": us,
           "road_slots_mean": float(counts[:, 0].mean()), "neighbour_slots_mean": float(counts[:, 1].mean()),
           "actor_critic_flop": flop,
           "actor_critic_tflops": flop / (us["actor_critic"] * 1e-6) / 1e12 if "actor_critic" in us else None,
           "actor_critic_frac_of_bf16_peak": (flop / (us["actor_critic"] * 1e-6) / 1e12 / BF16_PEAK_TFLOPS
                                              if "actor_critic" in us else None),
           "obs_full_gbs": obs_bytes_ / (us["obs_full"] * 1e-6) / 1e9 if "obs_full" in us else None}
    log(f"full observation + actor-critic on {workload}: {N} agents, {ms / steps:.4f} ms/step eager, "
        f"{out['casps_eager']:.4g} CASPS; kernels {us}")
    return out


def graph_len(steps: int) -> int:
    """Control steps per captured graph: the largest divisor of the timed
    step count up to 16, so that whole replays cover exactly that count."""
    return max(d for d in range(1, 17) if steps % d == 0)


def copy_bandwidth(torch, stream) -> float:
    """HBM bandwidth of a plain device-to-device copy (1 GiB read + 1 GiB
    written per copy), GB/s: the practical ceiling beside the 8 TB/s spec."""
    with torch.cuda.stream(stream):
        x = torch.empty(256 * 2 ** 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            y.copy_(x)
        e1.record(stream)
        torch.cuda.synchronize()
        gbs = 10 * 2 * x.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    return gbs


CLOCK_US = 50.0


def read_profile(sim, n_clock=20):
    """The handle's per-kernel event record, closed by `n_clock` kernels that
    run CLOCK_US of the GPU's constant-rate wall clock, timed the same way;
    returns ({kernel: (mean event us, launches)}, fixed us): an event pair
    bound to a dispatch still holds a fixed cost beside the kernel's
    execution, which the clock kernels measure (their mean less CLOCK_US)."""
    sim.profile_calibrate(n_clock, CLOCK_US)
    prof = sim.profile_read()
    sim.profile(False)
    t, c = prof.pop("clock")
    fixed = 1e3 * t / c - CLOCK_US if c else 0.0
    return {k: (1e3 * t / c, c) for k, (t, c) in prof.items() if c}, fixed


def kernel_us(ev, fixed):
    """Kernel means less the event pair's fixed cost."""
    return {k: us - fixed for k, (us, c) in ev.items()}


def measure(args, seed, torch, sf, I, stream, keep=False):
    """One seeded workload: warm-up, autotuned launch shapes, a profiled eager
    pass over the timed step count (per-kernel HIP events on the handle's
    stream), then the timed region: the same number of policy-driven control
    steps as replays of a captured graph."""
    worlds = I.workload(args.workload, seed=seed)
    dt, S = I.TIMING[args.workload]
    prm = dict(I.VEHICLE_DEFAULTS)
    policy = I.mlp_params([256, 256, 256, 2], seed=seed)
    K = args.steps
    with torch.cuda.stream(stream):
        sim = sf.Sim(worlds, prm, flags=sf.SF_AUTO_RESET, stream=stream, grid_cell=args.grid_cell,
                     obs_waves=args.obs_waves, step_block=args.step_block,
                     policy_rows=args.policy_rows)
        sim.policy_load(*policy)
        N = sim.N
        log(f"seed {seed}: {args.workload}: {worlds.num_worlds} worlds, {N} agents, "
            f"{len(worlds.road_xy)} road points, {len(worlds.tri_verts)} triangles")
        # the measured state is traffic SETTLE_STEPS control steps after spawn
        # (episodes running, contacts and resets in their steady mix), then
        # the requested warm-up
        for _ in range(SETTLE_STEPS + args.warmup):
            sim.step_policy(dt, S)
        torch.cuda.synchronize()
        tuning = sim.tuning()
        if not args.no_autotune:
            tuning = sim.autotune(dt, S, steps=args.tune_steps)
            log(f"autotuned: {tuning}")

        # profiled eager pass: per-kernel HIP events around every launch
        sim.profile(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(K):
            sim.step_policy(dt, S)
        e1.record(stream)
        torch.cuda.synchronize()
        eager_ms = e0.elapsed_time(e1)
        prof = read_profile(sim)

        # road data each kernel reads: distinct items per launch, counted in
        # the kernels over a separate eager pass (atomics on; not timed)
        sim.road_touch(True)
        for _ in range(TOUCH_STEPS):
            sim.step_policy(dt, S)
        items, tbytes, tsteps = sim.road_touch_read()
        sim.road_touch(False)
        road = {"step": float(tbytes[0]) / max(1, tsteps), "obs": float(tbytes[1]) / max(1, tsteps),
                "steps": int(tsteps)}

        # ---- timed region: K control steps as replays of a G-step graph
        G = graph_len(K)
        sim.graph_capture(G, dt, S)
        for _ in range(2):
            sim.graph_launch()
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record(stream)
        for _ in range(K // G):
            sim.graph_launch()
        g1.record(stream)
        torch.cuda.synchronize()
        ms = g0.elapsed_time(g1)
        f, k = sim.get_state()
        active = int(k[0].sum())
        # contact load where the timed region ended: overlapping vehicle pairs
        # in each substep of one more control step, taken by a second handle
        # that records its pair lists (the timed handle records none)
        probe = sf.Sim(worlds, prm, flags=sf.SF_AUTO_RESET | sf.SF_RECORD_CONTACTS, stream=stream)
        probe.policy_load(*policy)
        probe.set_state(f, k)
        probe.step_policy(dt, S)
        pairs = [int(probe.contacts(q)[0].sum()) for q in range(S)]
        probe.close()
    r = {"seed": seed, "road_bytes": road, "contact_pairs_per_substep": pairs, "casps": N * K / (ms / 1e3), "ms_per_step": ms / K, "graph_steps": G,
         "eager_casps": N * K / (eager_ms / 1e3), "eager_ms_per_step": eager_ms / K, "active": active,
         "N": N, "tuning": tuning, "prof": prof, "worlds": worlds, "prm": prm, "policy": policy,
         "dt": dt, "S": S}
    log(f"seed {seed}: graph {r['ms_per_step']:.4f} ms/step ({G}-step graphs), {r['casps']:.4g} CASPS; "
        f"eager {r['eager_ms_per_step']:.4f} ms/step; active {active}/{N}")
    if keep:
        r["sim"] = sim
    else:
        sim.close()
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--warmup", type=int, default=1500)
    ap.add_argument("--workload", default="uneven256")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--seeds", type=int, default=3, help="seeded workloads averaged (seed, seed+1, ...)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--sur-log-steps", type=int, default=50,
                    help="control steps of the benchmark workload logged as a second held-out set")
    ap.add_argument("--sur-train-samples", type=int, default=10_000_000)
    ap.add_argument("--grid-cell", type=float, default=0.0)
    ap.add_argument("--obs-waves", type=int, default=0)
    ap.add_argument("--step-block", type=int, default=0)
    ap.add_argument("--policy-rows", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tune-steps", type=int, default=20)
    ap.add_argument("--configs", default="cross1024x16,dense4096x32",
                    help="other workload sizes reported as context (empty: none)")
    ap.add_argument("--config-steps", type=int, default=300)
    ap.add_argument("--ppo-iters", type=int, default=2,
                    help="timed PPO iterations on the workload (0: no PPO leg)")
    ap.add_argument("--ppo-horizon", type=int, default=128)
    ap.add_argument("--full-obs-steps", type=int, default=100,
                    help="control steps of the paper-shaped observation + actor-critic leg (0: none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the step would shard by "
              "world across GPUs, and only the single-GPU step is implemented and measured", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.seeds < 1:
        print("--steps and --seeds must be >= 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_08528_amd import inputs as I, sf

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    copy_gbs = copy_bandwidth(torch, stream)
    log(f"device-to-device copy: {copy_gbs:.0f} GB/s")
    runs = [measure(args, args.seed + i, torch, sf, I, stream, keep=(i == 0)) for i in range(args.seeds)]
    r0 = runs[0]
    sim, N, tuning, prof = r0["sim"], r0["N"], r0["tuning"], r0["prof"]
    worlds, prm, policy, dt, S = r0["worlds"], r0["prm"], r0["policy"], r0["dt"], r0["S"]
    vals = np.array([r["casps"] for r in runs])
    value = float(vals.mean())
    ms = float(np.mean([r["ms_per_step"] for r in runs]))

    # ---- the same control step with the learned tire model inside (seed 0)
    sur = None
    if not args.no_surrogate:
        with torch.cuda.stream(stream):
            sur = surrogate_leg(sim, torch, sf, I, stream, dt, S, args.steps, min(args.warmup, 300),
                                args.sur_train_samples, args.sur_log_steps)

    # ---- the other workload sizes (context, not the headline value)
    others = {}
    if args.ppo_iters > 0:
        others["ppo_" + args.workload] = ppo_leg(torch, sf, I, stream, args.workload, args.ppo_horizon,
                                                 args.ppo_iters, args.seed)
        log(f"ppo on {args.workload}: {others['ppo_' + args.workload]['training_casps']:.4g} training CASPS "
            f"(rollout {others['ppo_' + args.workload]['rollout_ms']:.1f} ms, update "
            f"{others['ppo_' + args.workload]['update_ms']:.1f} ms per iteration)")
    if args.full_obs_steps > 0:
        others["full_obs_" + args.workload] = full_obs_leg(torch, sf, I, stream, args.workload,
                                                           args.full_obs_steps, args.seed)
    if args.configs:
        sur_params = None
        if sur is not None:
            with torch.cuda.stream(stream):
                sur_params = sim.sur_get()
        for name in [c for c in args.configs.split(",") if c]:
            others[name] = config_leg(name, torch, sf, I, stream, args.config_steps, sur_params,
                                      max(4, args.tune_steps // 2))

    ev, fixed = prof
    kernels = {name: {"avg_us": us - fixed, "event_us": us, "launches": cnt} for name, (us, cnt) in ev.items()}
    dom = max(kernels, key=lambda n: kernels[n]["avg_us"])
    avg_s = kernels[dom]["avg_us"] * 1e-6
    fused = tuning["obs_waves"] == 16
    road = r0["road_bytes"]
    if dom == "policy":
        flop = POLICY_FLOP_PER_AGENT * N
        roof = {"bound": "mfma", "achieved": flop / avg_s / 1e12, "peak": BF16_PEAK_TFLOPS,
                "unit": "TFLOP/s", "traffic": None}
    else:
        nbytes = step_bytes(N, road["step"]) if dom == "step" else obs_bytes(N, fused, road["obs"])
        roof = {"bound": "hbm", "achieved": nbytes / avg_s / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "traffic": None, "algorithmic_bytes": nbytes,
                "road_bytes": road["step"] if dom == "step" else road["obs"],
                "measured_copy_gbs": copy_gbs}
    roof["frac"] = roof["achieved"] / roof["peak"]
    launch = {"policy": "k_policy_lds<16>" if tuning["policy_rows"] <= 16 else f"k_policy<{tuning['policy_rows']}>",
              "step": f"k_step<{tuning['step_block']}, false>",
              "obs": "k_obs_policy" if fused else f"k_obs<{tuning['obs_waves']}>"}
    roof["kernel"] = launch[dom]
    roof["avg_us"] = kernels[dom]["avg_us"]
    roof["traffic"] = recorded_traffic({"policy": "k_policy", "step": "k_step", "obs": "k_obs"}[dom],
                                       launch[dom], N)
    roof["event_us"] = kernels[dom]["event_us"]
    roof["event_fixed_us"] = fixed
    roof["timing"] = ("mean HIP-event duration of the kernel (the event pair bound to its dispatch) over a "
                      "profiled eager pass of the same control steps, seed %d, less the event pair's fixed "
                      "cost: the mean event duration of a kernel that runs %.0f us of the GPU's wall clock, "
                      "less %.0f us" % (args.seed, CLOCK_US, CLOCK_US))
    # the whole control step (policy, step, observation) against the same peak
    whole = CONTROL_STEP_BYTES_PER_AGENT * N + POLICY_WEIGHT_BYTES + road["step"] + road["obs"]
    roof["control_step"] = {"algorithmic_bytes": whole, "ms": r0["ms_per_step"],
                            "achieved": whole / (r0["ms_per_step"] * 1e-3) / 1e9,
                            "frac": whole / (r0["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    for name in kernels:
        if name == "policy":
            kernels[name]["tflops"] = POLICY_FLOP_PER_AGENT * N / (kernels[name]["avg_us"] * 1e-6) / 1e12
        elif name in ("step", "obs"):
            nbytes = step_bytes(N, road["step"]) if name == "step" else obs_bytes(N, fused, road["obs"])
            kernels[name]["algorithmic_bytes"] = nbytes
            kernels[name]["algorithmic_gbs"] = nbytes / (kernels[name]["avg_us"] * 1e-6) / 1e9
            if name == "obs" and fused:
                kernels[name]["policy_tflops"] = POLICY_FLOP_PER_AGENT * N / (kernels[name]["avg_us"] * 1e-6) / 1e12

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(worlds, prm, float(np.float32(dt)), S, policy, args.cpu_seconds)
        log(f"cpu oracle: {cpu['value']:.4g} CASPS on {cpu['cores']} threads")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "controlled-agent steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {worlds.num_worlds} worlds, {N} agents "
                        f"({int(np.diff(worlds.agent_offsets).min())}-{int(np.diff(worlds.agent_offsets).max())} per world), "
                        f"{len(worlds.road_xy)} road points, dt {dt:.4f} s x {S} substeps, "
                        "plain tire, policy MLP 256-256-256-2 bf16/fp32-acc",
            "step": ("physics step + observation with the next actions in the same kernel"
                     if fused else "policy + physics step + observation"),
            "timed": f"{args.steps} control steps as replays of {r0['graph_steps']}-step hipGraphs, "
                     f"mean over seeds {[r['seed'] for r in runs]}",
            "active_agents": r0["active"],
            "settle_steps": SETTLE_STEPS,
            "contact_pairs_per_substep_after_timed": r0["contact_pairs_per_substep"],
            "launch_shapes": {k: tuning[k] for k in ("step_block", "step_grid", "obs_waves", "policy_rows")},
        },
        "value_stdev": float(vals.std(ddof=1)) if len(runs) > 1 else 0.0,
        "seeds": [{"seed": r["seed"], "casps": r["casps"], "ms_per_step": r["ms_per_step"],
                   "eager_casps": r["eager_casps"],
                   "launch_shapes": {k: r["tuning"][k] for k in ("step_block", "step_grid", "obs_waves",
                                                                  "policy_rows")}} for r in runs],
        "eager": {"casps": float(np.mean([r["eager_casps"] for r in runs])),
                  "ms_per_step": float(np.mean([r["eager_ms_per_step"] for r in runs])),
                  "note": "one launch per kernel from the host, per-kernel events on"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "surrogate": sur,
        "other_configs": others,
        "paper_context": {"casps": 19250, "hardware": "RTX PRO 6000 Blackwell, PhysX, 256x16"},
    }
    print(json.dumps(out))
    sim.close()


if __name__ == "__main__":
    main()
