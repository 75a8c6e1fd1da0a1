"""Pins of the oracle's paper-shaped observation and late-fusion actor-critic
(appendix "Observation Space Details", appendix "Network Architecture
Details"), on the CPU: dimensions fixed by the paper, known answers on
hand-built roads, and the network against torch's float64 layers."""
import math

import numpy as np
import pytest
import torch

from tests.helpers import params, world

EGO, RK, VK = 11, 350, 24


@pytest.fixture(scope="module")
def O(oracle_mod):
    return oracle_mod


def test_observation_dimension_and_parameter_count(O):
    # 7 ego + 4 weather, 350 road points x 5, 24 neighbours x 7
    assert O.FULL_DIM == 1929 == 7 + 4 + 350 * 5 + 24 * 7
    # per network: encoders 11-64-64, 5-96-96, 7-96-96, trunk 256-128-64
    body = (11 * 64 + 64) + (64 * 64 + 64) + (5 * 96 + 96) + (96 * 96 + 96) + (7 * 96 + 96) + (96 * 96 + 96) \
        + (256 * 128 + 128) + (128 * 64 + 64)
    assert O.AC_PARAMS == 2 * body + (3 * 64 + 3) + 3 + (64 + 1)


def _line_world(yaw, n=200, spacing=0.5, agents=None):
    """Road points on the x axis from x = -50 m every 0.5 m (type 2, along
    +x) and one agent at the origin heading `yaw`, goal 30 m ahead."""
    xs = -50.0 + spacing * np.arange(n)
    road = np.stack([xs, np.zeros(n)], 1).astype(np.float32)
    gx, gy = 30 * math.cos(yaw), 30 * math.sin(yaw)
    sp = [(0.0, 0.0, yaw, gx, gy)] + (agents or [])
    w = world(sp, road_xy=road)
    w.road_dir = np.tile(np.array([[1.0, 0.0]], np.float32), (n, 1))
    return w


def test_road_slots_within_ten_metres_in_index_order(O):
    """41 points lie within 10 m (x = -10 .. 10, both ends inclusive); in
    index order they run from x = -10 to +10; body-frame features rotate
    with the heading."""
    for yaw in (0.0, math.pi / 2):
        o = O.Oracle(_line_world(yaw), params())
        obs, cnt = o.observe_full()
        assert cnt[0, 0] == 41 and cnt[0, 1] == 0
        r = obs[0, EGO:EGO + 5 * RK].reshape(RK, 5)
        x = -10.0 + 0.5 * np.arange(41)
        c, s = math.cos(np.float32(yaw)), math.sin(np.float32(yaw))
        # body frame: (c x, -s x) / 10; direction (1, 0) -> (c, -s)
        assert np.allclose(r[:41, 0], c * x / 10, atol=1e-6) and np.allclose(r[:41, 1], -s * x / 10, atol=1e-6)
        assert np.allclose(r[:41, 2], 2 / 20) and np.allclose(r[:41, 3], c, atol=1e-6)
        assert np.allclose(r[:41, 4], -s, atol=1e-6)
        assert not r[41:].any()
        idx, n = o.road_within(0)
        assert n == 41 and list(idx[:41]) == list(range(80, 121))


def test_road_slots_truncate_to_the_first_350_by_index(O):
    """A 41 x 41 lattice at 0.5 m around the agent holds 1257 points within
    10 m; the observation keeps the 350 lowest indices (row-major, so the
    first rows of the disc), not the nearest ones."""
    g = -10.0 + 0.5 * np.arange(41)
    X, Y = np.meshgrid(g, g)               # row-major: y outer, x inner
    road = np.stack([X.ravel(), Y.ravel()], 1).astype(np.float32)
    w = world([(0.0, 0.0, 0.0, 30.0, 0.0)], road_xy=road)
    w.road_dir = np.tile(np.array([[0.0, 1.0]], np.float32), (len(road), 1))
    o = O.Oracle(w, params())
    obs, cnt = o.observe_full()
    inside = np.nonzero(X.ravel() ** 2 + Y.ravel() ** 2 <= 100.0 + 1e-9)[0]
    assert len(inside) == 1257
    assert cnt[0, 0] == 350
    idx, n = o.road_within(0)
    assert list(idx[:350]) == list(inside[:350])
    r = obs[0, EGO:EGO + 5 * RK].reshape(RK, 5)
    assert np.allclose(r[:, 0] * 10, X.ravel()[inside[:350]], atol=1e-5)
    assert np.allclose(r[:, 1] * 10, Y.ravel()[inside[:350]], atol=1e-5)


def test_ego_and_weather_token(O):
    """Goal 30 m ahead at 45 degrees to the left of the heading: body-frame
    goal (21.2, 21.2)/100, bearing sine and cosine 1/sqrt 2, distance 0.3;
    weather token (film / 1 mm, one-hot pavement) per world."""
    yaw = 0.3
    w = _line_world(yaw)
    g = 30.0 / math.sqrt(2)
    a = yaw + math.pi / 4
    w.spawn[0, 3:5] = (30 * math.cos(a), 30 * math.sin(a))
    for pav in (0, 1, 2):
        w.film_mm[:] = 0.37
        w.pavement[:] = pav
        o = O.Oracle(w, params())
        obs, _ = o.observe_full()
        e = obs[0, :EGO]
        assert np.allclose(e[:2], g / 100, atol=2e-6)
        assert np.allclose(e[2:4], 1 / math.sqrt(2), atol=1e-6) and abs(e[4] - 0.3) < 1e-6
        assert np.allclose(e[5:7], 0.0)
        assert abs(e[7] - np.float32(0.37)) < 1e-7
        onehot = np.zeros(3, np.float32)
        onehot[pav] = 1
        assert np.array_equal(e[8:11], onehot)


def test_neighbours_24_nearest_ascending(O):
    """30 other vehicles 3 m apart along a line behind and ahead: the 24
    nearest, ascending, features at 1/100 scale; the rest are left out."""
    others = [(3.0 * k * (1 if k % 2 else -1), 5.0, 0.0, 0.0, 0.0) for k in range(1, 31)]
    w = _line_world(0.0, agents=others)
    o = O.Oracle(w, params())
    # place every vehicle explicitly (the spawn rotation may permute entries)
    f, k = o.get_state()
    f[0], f[1] = [0.0] + [e[0] for e in others], [0.0] + [e[1] for e in others]
    f[3], f[4], f[5], f[6] = 1.0, 0.0, 0.0, 0.0
    o.set_state(f, k)
    obs, cnt = o.observe_full()
    assert cnt[0, 1] == 24
    d = np.hypot([e[0] for e in others], 5.0)
    order = np.argsort(d, kind="stable")[:24] + 1
    assert list(o.knn_neigh_k(0)) == list(order)
    v = obs[0, EGO + 5 * RK:].reshape(VK, 7)
    for k, j in enumerate(order):
        ex, ey = others[j - 1][0], others[j - 1][1]
        assert abs(v[k, 0] - ex / 100) < 1e-6 and abs(v[k, 1] - ey / 100) < 1e-6
        assert abs(v[k, 2] - 0.04) < 1e-7 and abs(v[k, 3] - 0.02) < 1e-7


# ------------------------------------------------------- actor-critic
def _torch_ac(P, obs, counts):
    """The same architecture from torch's float64 layers."""
    P = torch.from_numpy(P.astype(np.float64))
    off = [0]

    def lin(i, o):
        W = P[off[0]:off[0] + i * o].reshape(o, i)
        b = P[off[0] + i * o:off[0] + i * o + o]
        off[0] += i * o + o
        lay = torch.nn.Linear(i, o, dtype=torch.float64)
        with torch.no_grad():
            lay.weight.copy_(W)
            lay.bias.copy_(b)
        return lay

    elu = torch.nn.ELU()
    nets = []
    for head in (3, 1):
        net = {"e": [lin(11, 64), lin(64, 64)], "r": [lin(5, 96), lin(96, 96)], "v": [lin(7, 96), lin(96, 96)],
               "t": [lin(256, 128), lin(128, 64)], "h": lin(64, head)}
        if head == 3:
            off[0] += 3          # log sigma
        nets.append(net)
    x = torch.from_numpy(obs.astype(np.float64))
    outs = []
    for net in nets:
        e = elu(net["e"][1](elu(net["e"][0](x[:, :11]))))
        rr = x[:, 11:11 + 5 * RK].reshape(-1, RK, 5)
        vv = x[:, 11 + 5 * RK:].reshape(-1, VK, 7)
        pools = []
        for seq, key, cidx in ((rr, "r", 0), (vv, "v", 1)):
            z = elu(net[key][1](elu(net[key][0](seq))))
            mask = torch.arange(seq.shape[1])[None, :] < torch.from_numpy(counts[:, cidx])[:, None]
            z = torch.where(mask[:, :, None], z, torch.tensor(-math.inf, dtype=torch.float64))
            pool = z.max(dim=1).values
            pool = torch.where(torch.isinf(pool), torch.zeros_like(pool), pool)
            pools.append(pool)
        t = elu(net["t"][1](elu(net["t"][0](torch.cat([e] + pools, 1)))))
        outs.append(net["h"](t))
    assert off[0] == P.numel()
    return outs[0].detach().numpy(), outs[1][:, 0].detach().numpy()


def _random_ac_inputs(O, M, seed):
    rng = np.random.default_rng(seed)
    P = (rng.standard_normal(O.AC_PARAMS) * 0.15).astype(np.float32)
    obs = rng.uniform(-1, 1, (M, O.FULL_DIM)).astype(np.float32)
    counts = np.stack([rng.integers(0, RK + 1, M), rng.integers(0, VK + 1, M)], 1).astype(np.int32)
    counts[0] = (0, 0)
    counts[1] = (RK, VK)
    return P, obs, counts


def test_actor_critic_matches_torch_float64(O):
    """With the bf16 rounding points off, the oracle is the plain float64
    network: masked max-pool over the valid slots, empty sets pool to 0."""
    P, obs, counts = _random_ac_inputs(O, 12, 3)
    O.set_bf16(False)
    try:
        m, v = O.actor_critic(P, obs, counts)
    finally:
        O.set_bf16(True)
    mt, vt = _torch_ac(P, obs, counts)
    assert np.allclose(m, mt, rtol=1e-10, atol=1e-10)
    assert np.allclose(v, vt, rtol=1e-10, atol=1e-10)


def test_actor_critic_ignores_padding_and_rounds_to_bf16(O):
    """Values in slots past the counts change nothing; with the rounding
    points on, the outputs move by about the bf16 quantum only."""
    P, obs, counts = _random_ac_inputs(O, 8, 4)
    m0, v0 = O.actor_critic(P, obs, counts)
    obs2 = obs.copy().reshape(8, -1)
    for r in range(8):
        road = obs2[r, 11:11 + 5 * RK].reshape(RK, 5)
        road[counts[r, 0]:] = 7.0
        veh = obs2[r, 11 + 5 * RK:].reshape(VK, 7)
        veh[counts[r, 1]:] = -3.0
    m1, v1 = O.actor_critic(P, obs2, counts)
    assert np.array_equal(m0, m1) and np.array_equal(v0, v1)
    mt, vt = _torch_ac(P, obs, counts)
    scale = max(np.abs(mt).max(), np.abs(vt).max())
    assert np.abs(m0 - mt).max() < 0.05 * scale and np.abs(m0 - mt).max() > 0.0
