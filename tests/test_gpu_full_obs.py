"""The paper-shaped observation and the late-fusion actor-critic through the
C ABI against the FP64 oracle.

* observation: valid slot counts bit for bit; every feature within 1e-4
  (road slots in point-index order and neighbour order follow from integer
  keys, so a membership slip shows up as a gross feature mismatch), except a
  time to collision whose definition sits on a threshold on the shared state
  (checked in FP64) and the relative heading's +-1 wrap;
* network: mean and value against the oracle with the same bf16 rounding
  points, relative norm <= 1e-2 and elementwise bounds, on ragged batches
  (a partial 16-agent tile, inactive agents, empty and full sets);
* the step driven by the network's actions matches the oracle's step on the
  same actions.
"""
import numpy as np
import pytest

from paper_2605_08528_amd import inputs as I
from tests.helpers import params as mkparams, ttc_explained, world
from tests.test_gpu_parity import GROUPS, TOL, _at_speed, cuda, make_pair, rel_err, seed_oracle

pytestmark = pytest.mark.gpu

EGO, RK, VK = 11, 350, 24
DIM = EGO + 5 * RK + 7 * VK


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a GPU"
    return T


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as O
    O.build()
    return O


def lattice_world(seed=0):
    """A dense 0.5 m lattice of road points around several vehicles: more
    than 350 points within 10 m of each, so the index-order truncation
    decides."""
    g = -12.0 + 0.5 * np.arange(49)
    X, Y = np.meshgrid(g, g)
    road = np.stack([X.ravel(), Y.ravel()], 1).astype(np.float32)
    sp = [(-4.0, 0.0, 0.3, 30.0, 0.0), (4.0, 2.0, -1.0, -30.0, 0.0), (0.0, -6.0, 2.0, 0.0, 30.0)]
    w = world(sp, road_xy=road)
    ang = np.random.default_rng(seed).uniform(0, 2 * np.pi, len(road))
    w.road_dir = np.stack([np.cos(ang), np.sin(ang)], 1).astype(np.float32)
    w.road_type = (np.arange(len(road)) % 20).astype(np.uint8)
    w.film_mm[:] = 0.42
    w.pavement[:] = 2
    return w


def compare_full_obs(O, fg, kg, og, cg, oo, co, prm, worlds):
    """Feature-by-feature comparison; returns the number of explained TTC entries."""
    assert np.array_equal(cg, co)
    d = np.abs(og.astype(np.float64) - oo.astype(np.float64))
    veh = d[:, EGO + 5 * RK:].reshape(-1, VK, 7)
    vg = og[:, EGO + 5 * RK:].reshape(-1, VK, 7)
    # relative heading: +1 and -1 are the same angle
    veh[:, :, 4] = np.minimum(veh[:, :, 4], 2.0 - veh[:, :, 4])
    explained = 0
    cr, cd = O.circle_model(prm)
    ao = worlds.agent_offsets
    orc_idx = {}
    for r, s in np.argwhere(veh[:, :, 6] > 1e-4):
        w = int(np.searchsorted(ao, r, side="right") - 1)
        if r not in orc_idx:
            orc_idx[r] = O_knn(O, worlds, prm, fg, kg, r)
        j = int(ao[w]) + int(orc_idx[r][s])
        ok, _ = ttc_explained(fg.astype(np.float64), r, j, cr, cd, 10.0 * float(vg[r, s, 6]))
        assert ok, (r, s)
        veh[r, s, 6] = 0.0
        explained += 1
    worst = d.max() if d.size else 0.0
    assert worst < 1e-4, (worst, np.unravel_index(d.argmax(), d.shape))
    return explained


def O_knn(O, worlds, prm, f, k, r):
    o = O.Oracle(worlds, prm)
    o.set_state(f.astype(np.float64), k)
    return o.knn_neigh_k(r)


@pytest.mark.parametrize("case", ["cross", "uneven", "lattice"])
def test_full_observation_matches_oracle(O, torch, case):
    from paper_2605_08528_amd import sf
    if case == "cross":
        w = I.intersections(12, 16, seed=21, rain=True)
        w.pavement[:] = np.arange(12) % 3
    elif case == "uneven":
        w = I.uneven_manhattan(6, agents=(4, 32), points=(1000, 6000), seed=22, mean_agents=16)
    else:
        w = lattice_world()
    prm = mkparams()
    sim, orc = make_pair(O, torch, w, prm)
    f, k = sim.get_state()
    _at_speed(23, 2.0, 12.0)(f, k)
    if case == "cross":
        k[0, ::7] = 0                      # some inactive agents
    sim.set_state(f, k)
    for step in range(3):
        sim.step(cuda(torch, I.actions(23, step, sim.N)), 1.0 / 30.0, 4)
    obs, cnt = sim.observe_full()
    torch.cuda.synchronize()
    fg, kg = sim.get_state()
    seed_oracle(orc, sim)
    oo, co = orc.observe_full()
    og, cg = obs.cpu().numpy(), cnt.cpu().numpy()
    n_expl = compare_full_obs(O, fg, kg, og, cg, oo, co, prm, w)
    print(case, "agents", sim.N, "road slots mean", cg[:, 0].mean(), "max", cg[:, 0].max(),
          "neighbours mean", cg[:, 1].mean(), "explained TTC", n_expl)
    if case == "lattice":
        assert (cg[:, 0] == RK).all()
        assert np.allclose(og[:, 7], 0.42) and (og[:, 10] == 1).all()
    sim.close()


def ac_params(O, seed, scale=0.12):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(O.AC_PARAMS) * scale).astype(np.float32)


def test_actor_critic_matches_oracle(O, torch):
    """MFMA encoders, masked max-pools and trunk against the FP64 network
    with the same bf16 rounding points, on observations from the GPU; the
    batch has a partial 16-agent tile, inactive agents and full sets."""
    from paper_2605_08528_amd import sf
    for w in (I.intersections(9, 13, seed=24), lattice_world(1)):
        sim, orc = make_pair(O, torch, w, mkparams())
        f, k = sim.get_state()
        _at_speed(24, 2.0, 12.0)(f, k)
        k[0, ::5] = 0
        sim.set_state(f, k)
        P = ac_params(O, 7)
        sim.actor_critic_load(P)
        obs, cnt = sim.observe_full()
        mean, value = sim.actor_critic(obs, cnt)
        torch.cuda.synchronize()
        m_g, v_g = mean.cpu().numpy().astype(np.float64), value.cpu().numpy().astype(np.float64)
        m_o, v_o = O.actor_critic(P, obs.cpu().numpy(), cnt.cpu().numpy())
        for name, g, o in (("mean", m_g, m_o), ("value", v_g, v_o)):
            rel = np.linalg.norm(g - o) / np.linalg.norm(o)
            mx = np.abs(g - o).max()
            print(w.name, name, "relative error", rel, "max abs", mx, "scale", np.abs(o).max())
            assert rel <= 1e-2
            assert mx <= 2e-2 * max(1.0, np.abs(o).max())
        sim.close()


def test_step_actor_critic_matches_oracle(O, torch):
    """One control step driven by the network: the actions decode the mean
    (throttle and brake rectified, steering clamped and scaled), and the
    step on them matches the oracle's step on the same actions."""
    w = I.intersections(8, 8, seed=25)
    prm = mkparams()
    sim, orc = make_pair(O, torch, w, prm)
    f, k = sim.get_state()
    _at_speed(25, 3.0, 10.0)(f, k)
    sim.set_state(f, k)
    P = ac_params(O, 8, scale=0.3)
    sim.actor_critic_load(P)
    for step in range(4):
        seed_oracle(orc, sim)
        sim.step_actor_critic(1.0 / 30.0, 4)
        mean, value, act, obs, cnt = sim.actor_critic_read()
        torch.cuda.synchronize()
        m = mean.cpu().numpy()
        a = act.cpu().numpy()
        thr = np.clip(m[:, 0], 0, 1)
        brk = np.clip(m[:, 2], 0, 1)
        str_ = np.clip(m[:, 1], -1, 1)
        assert np.array_equal(a[:, 0], (thr - brk).astype(np.float32))
        assert np.array_equal(a[:, 1], (np.float32(0.5) * str_).astype(np.float32))
        assert np.abs(a[:, 0]).max() > 0.0
        orc.step(a, float(np.float32(1.0 / 30.0)), 4)
        fg, kg = sim.get_state()
        fo, ko = orc.get_state()
        err = rel_err(fg, fo)
        assert all(err[g] <= TOL for g in GROUPS), (step, err)
        assert np.array_equal(kg, ko)
    sim.close()
