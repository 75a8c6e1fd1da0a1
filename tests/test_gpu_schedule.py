"""Uneven batching: the persistent world queue and the launch-shape
autotuner, through the C ABI.

* a persistent grid smaller than the number of worlds (workgroups pull worlds,
  largest first, from an atomic queue) gives bitwise the same states as one
  workgroup per world, in eager launches and in replays of a captured graph
  (the queue re-arms itself inside the kernel), and matches the oracle in
  lockstep;
* the autotuner returns valid shapes with their measured times, leaves the
  simulation state exactly as it found it, and a second handle with the same
  workload takes the cached choice without measuring.
"""
import numpy as np
import pytest

from paper_2605_08528_amd import inputs as I
from tests.helpers import params as mkparams
from tests.test_gpu_parity import lockstep, cuda, O, torch  # noqa: F401 (fixtures)

pytestmark = pytest.mark.gpu


def run(torch, worlds, steps, graph=False, **kw):
    from paper_2605_08528_amd import sf
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim = sf.Sim(worlds, mkparams(), flags=sf.SF_AUTO_RESET, stream=stream, **kw)
        sim.policy_load(*I.mlp_params([256, 256, 256, 2], seed=3))
        dt, S = 1.0 / 30.0, 4
        out = []
        if graph:
            sim.graph_capture(4, dt, S)
            for _ in range(steps // 4):
                sim.graph_launch()
                torch.cuda.synchronize()
                out.append(sim.get_state())
        else:
            for k in range(steps):
                sim.step_policy(dt, S)
                if k % 4 == 3:
                    torch.cuda.synchronize()
                    out.append(sim.get_state())
        obs = sim.observe()[0].cpu().numpy()
        sim.close()
    return out, obs


def test_persistent_queue_bitwise_equal(torch):
    w = I.workload("uneven256")
    ref, obs_ref = run(torch, w, 24)
    for grid, graph in ((40, False), (7, False), (40, True)):
        got, obs = run(torch, w, 24, graph=graph, step_grid=grid)
        for (fa, ka), (fb, kb) in zip(got, ref):
            assert np.array_equal(fa, fb) and np.array_equal(ka, kb), (grid, graph)
        assert np.array_equal(obs, obs_ref)


def test_persistent_queue_lockstep(O, torch):
    w = I.intersections(16, 8, seed=5)
    dt, S = I.TIMING["cross64x8"]
    worst, _ = lockstep(O, torch, w, 30, dt, S, step_grid=3)
    print("persistent (3 workgroups, 16 worlds) worst relative error", worst)


def test_autotune_restores_state_and_caches(torch, tmp_path):
    from paper_2605_08528_amd import sf
    w = I.workload("uneven256")
    dt, S = I.TIMING["uneven256"]
    cache = str(tmp_path / "tune.txt")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim = sf.Sim(w, mkparams(), flags=sf.SF_AUTO_RESET, stream=stream)
        sim.policy_load(*I.mlp_params([256, 256, 256, 2], seed=0))
        for _ in range(30):
            sim.step_policy(dt, S)
        torch.cuda.synchronize()
        f0, k0 = sim.get_state()
        obs0 = sim.observe()[0].cpu().numpy()
        t = sim.autotune(dt, S, steps=4, cache_path=cache)
        f1, k1 = sim.get_state()
        obs1 = sim.observe()[0].cpu().numpy()
        assert np.array_equal(f0, f1) and np.array_equal(k0, k1) and np.array_equal(obs0, obs1)
        assert t["step_block"] in (64, 128, 192, 256, 320) and t["obs_waves"] in (1, 2, 4, 16)
        assert t["policy_rows"] in (16, 32, 64) and t["step_grid"] >= 0
        assert t["grid_cell"] in (4.0, 8.0, 16.0) and t["tri_cell"] in (0.5, 1.0)
        assert t["step_us"] > 0 and t["obs_us"] > 0
        # the fused observation leaves no policy launch to time
        assert (t["policy_us"] > 0) != (t["obs_waves"] == 16)
        assert sim.tuning()["step_block"] == t["step_block"]
        print("autotuned shapes", t)
        # the chosen shapes step on as usual
        sim.step_policy(dt, S)
        sim.close()
        lines = open(cache).read().splitlines()
        assert len(lines) == 1 and lines[0].startswith("W256 N4096")
        sim2 = sf.Sim(w, mkparams(), flags=sf.SF_AUTO_RESET, stream=stream)
        t2 = sim2.autotune(dt, S, steps=4, cache_path=cache)
        keys = ("step_block", "step_grid", "obs_waves", "policy_rows", "grid_cell", "tri_cell")
        assert {k: t2[k] for k in keys} == {k: t[k] for k in keys}
        assert t2["step_us"] == 0.0          # taken from the cache, not measured
        with pytest.raises(sf.SFError):
            sim2.set_tuning(100, 0, 4, 16)
        sim2.close()


def test_grid_cells_leave_results_unchanged(torch):
    """Rebuilding a handle's grids with other cell sizes changes only the
    cost: the exact kNN and the wheel rays give bitwise the same states,
    events and observations; a captured graph, which holds the old grids, is
    dropped."""
    from paper_2605_08528_amd import sf
    w = I.workload("cross64x8")
    dt, S = I.TIMING["cross64x8"]
    out = []
    for gc, tc in ((8.0, 0.5), (4.0, 1.0), (16.0, 0.25), (2.0, 0.5)):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            sim = sf.Sim(w, mkparams(), flags=sf.SF_AUTO_RESET, stream=stream)
            sim.policy_load(*I.mlp_params([256, 256, 256, 2], seed=3))
            sim.graph_capture(2, dt, S)
            t = sim.tuning()
            sim.set_tuning(t["step_block"], t["step_grid"], t["obs_waves"], t["policy_rows"], gc, tc)
            t2 = sim.tuning()
            assert (t2["grid_cell"], t2["tri_cell"]) == (gc, tc)
            if (gc, tc) != (8.0, 0.5):
                with pytest.raises(sf.SFError):
                    sim.graph_launch()
            for step in range(8):
                sim.step(cuda(torch, I.actions(31, step, sim.N)), dt, S)
            obs, rew, done, ev = sim.observe()
            torch.cuda.synchronize()
            f, k = sim.get_state()
            out.append((f.view(np.uint32).copy(), k.copy(), obs.cpu().numpy().view(np.uint32),
                        ev.cpu().numpy(), sim.debug_obs_indices()))
            sim.close()
    names = ("state", "integer state", "observation", "events", "kNN indices")
    cfgs = ((8.0, 0.5), (4.0, 1.0), (16.0, 0.25), (2.0, 0.5))
    bad = []
    for c, o in zip(cfgs[1:], out[1:]):
        for nm, a, b in zip(names, out[0], o):
            if not np.array_equal(a, b):
                cols = np.nonzero((a != b).reshape(a.shape[0], -1).any(axis=0) if nm == "state"
                                  else (a != b).reshape(a.shape[0], -1).any(axis=1))[0]
                bad.append((c, nm, len(cols), cols[:8].tolist()))
    assert not bad, bad
