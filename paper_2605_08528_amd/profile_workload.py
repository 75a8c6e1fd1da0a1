"""A short, fixed sequence of the library's kernels for counter collection.

    python3 -m paper_2605_08528_amd.profile_workload [--workload uneven256] [--steps 20]

Under ``rocprofv3 --pmc ...`` every dispatch is serialised and counted, so
the sequence stays short: a 256 MiB device copy (the calibration of the
memory counters against a transfer of known size), the workload settled for
``--settle`` policy-driven control steps, then ``--steps`` control steps with
the plain step and the fused observation + policy kernel, the same number
with the policy, step and observation kernels launched separately, a learned tire model fitted briefly on samples logged
from the plain step (``--train-steps`` Adam steps of the training kernels),
``--steps`` control steps with the network inside the step, and ``--steps``
control steps driven by the paper-shaped observation and the late-fusion
actor-critic (seeded random weights), one short PPO iteration (a 4-step
rollout, one epoch of two minibatches), and last ``--steps`` fused control
steps at each step workgroup shape of ``--step-blocks``.  Launch shapes are
fixed (no autotuning) so that the kernels are the ones named on the command
line.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="uneven256")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--settle", type=int, default=300)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--train-steps", type=int, default=200)
    ap.add_argument("--step-block", type=int, default=192)
    ap.add_argument("--obs-waves", type=int, default=16)
    ap.add_argument("--policy-rows", type=int, default=16)
    ap.add_argument("--step-blocks", default="64,128,192,256,320")
    args = ap.parse_args()

    import torch
    from paper_2605_08528_amd import inputs as I, sf

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        x = torch.empty(64 * 2 ** 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
        w = I.workload(args.workload, seed=args.seed)
        dt, S = I.TIMING[args.workload]
        sim = sf.Sim(w, dict(I.VEHICLE_DEFAULTS), flags=sf.SF_AUTO_RESET, stream=stream,
                     step_block=args.step_block, obs_waves=args.obs_waves, policy_rows=args.policy_rows)
        sim.policy_load(*I.mlp_params([256, 256, 256, 2], seed=args.seed))
        for _ in range(args.settle):
            sim.step_policy(dt, S)
        torch.cuda.synchronize()
        print(f"profile_workload: {args.workload}, {sim.N} agents, settled {args.settle} steps", file=sys.stderr,
              flush=True)
        for _ in range(args.steps):
            sim.step_policy(dt, S)
        # the unfused path: policy kernel, step, observation kernel
        sim.set_tuning(args.step_block, 0, 4, args.policy_rows)
        for _ in range(args.steps):
            sim.step_policy(dt, S)
        sim.set_tuning(args.step_block, 0, args.obs_waves, args.policy_rows)
        torch.cuda.synchronize()
        cap = 50 * S * 4 * sim.N
        sim.sur_log(cap)
        for _ in range(50):
            sim.step_policy(dt, S)
        data, n = sim.sur_collect(cap)
        sim.sur_log(0)
        sim.sur_fit(data, schedule=((2e-3, args.train_steps),))
        sim.sur_enable(True)
        for _ in range(args.steps):
            sim.step_policy(dt, S)
        torch.cuda.synchronize()
        used, fb = sim.sur_counts()
        sim.sur_enable(False)
        # the paper-shaped observation and the late-fusion actor-critic
        rng = np.random.default_rng(args.seed)
        sim.actor_critic_load((rng.standard_normal(sf.AC_PARAMS) * 0.1).astype(np.float32))
        for _ in range(args.steps):
            sim.step_actor_critic(dt, S)
        torch.cuda.synchronize()
        # one short PPO iteration: a 4-step rollout, one epoch of two
        # minibatches (training forward pass, loss, backward pass, Adam)
        opts = sim.ppo_init(horizon=4, epochs=1, minibatches=2)
        g = torch.Generator(device="cuda").manual_seed(args.seed)
        eps = torch.randn((4, sim.N, 3), generator=g, device="cuda", dtype=torch.float32)
        perm = torch.randperm(4 * sim.N, generator=g, device="cuda").to(torch.int32)[None]
        sim.ppo_rollout(eps, dt, S)
        sim.ppo_update(perm)
        torch.cuda.synchronize()
        # last: the fused policy-driven step at every step workgroup shape, so
        # that each shape's last dispatches are its own control steps
        for block in [int(b) for b in args.step_blocks.split(",") if b]:
            sim.set_tuning(block, 0, args.obs_waves, args.policy_rows)
            for _ in range(args.steps):
                sim.step_policy(dt, S)
        torch.cuda.synchronize()
        sim.close()
    print(json.dumps({"workload": args.workload, "agents": sim.N, "steps": args.steps, "samples": int(n),
                      "network_wheel_substeps": used, "fallback_wheel_substeps": fb}))


if __name__ == "__main__":
    main()
