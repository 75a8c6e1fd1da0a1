"""The seeded synthetic workloads have the shapes the benchmark and the
parity tests rely on: world and agent counts, per-world ranges, road types,
triangle strips, spawn tables, friction classes and seed determinism."""
import numpy as np
import pytest

from paper_2605_08528_amd import inputs as I


def check_csr(off, total):
    assert off[0] == 0 and off[-1] == total
    assert np.all(np.diff(off) >= 0)


def check_worlds(w):
    W = w.num_worlds
    for off in (w.agent_offsets, w.road_offsets, w.tri_offsets, w.spawn_offsets):
        assert off.shape == (W + 1,)
    check_csr(w.agent_offsets, w.num_agents)
    check_csr(w.road_offsets, len(w.road_xy))
    check_csr(w.tri_offsets, len(w.tri_verts))
    check_csr(w.spawn_offsets, len(w.spawn))
    assert w.road_xy.dtype == np.float32 and w.tri_verts.shape[1:] == (3, 3)
    assert set(np.unique(w.road_type)) <= {I.ROAD_LANE, I.ROAD_EDGE_LEFT, I.ROAD_EDGE_RIGHT}
    # flat roads (z-flattened) and non-degenerate triangles
    assert np.all(w.tri_verts[:, :, 2] == 0.0)
    e1 = w.tri_verts[:, 1, :2] - w.tri_verts[:, 0, :2]
    e2 = w.tri_verts[:, 2, :2] - w.tri_verts[:, 0, :2]
    assert np.all(np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]) > 1e-3)
    assert w.tri_surface.max() < w.num_surfaces
    assert w.mu_class.shape == (W, w.num_surfaces)
    # every world has at least as many spawn entries as agents, goals 3-100 m+ away
    assert np.all(np.diff(w.spawn_offsets) >= np.diff(w.agent_offsets))
    if len(w.spawn):
        d = np.hypot(w.spawn[:, 3] - w.spawn[:, 0], w.spawn[:, 4] - w.spawn[:, 1])
        assert d.min() >= 3.0


def test_uneven256_shape():
    """256 worlds, 4-32 vehicles each, 4096 in total, 1k-20k road points."""
    w = I.workload("uneven256")
    check_worlds(w)
    a = np.diff(w.agent_offsets)
    p = np.diff(w.road_offsets)
    assert w.num_worlds == 256 and w.num_agents == 4096
    assert a.min() >= 4 and a.max() <= 32 and a.max() > 24 and a.min() < 8
    assert p.min() >= 1000 and p.max() <= 20500 and p.max() > 10000
    assert set(np.unique(w.mu_class)) <= set(I.MU_CLASSES.tolist())


def test_cross64x8_shape():
    w = I.workload("cross64x8")
    check_worlds(w)
    assert w.num_worlds == 64 and np.all(np.diff(w.agent_offsets) == 8)
    p = np.diff(w.road_offsets)
    assert np.all((p > 1500) & (p < 2600))


def test_road_points_spaced_half_a_metre():
    """Consecutive points of one polyline are 0.5 m apart."""
    w = I.workload("cross64x8").world_slice(0, 1)
    d = np.hypot(*np.diff(w.road_xy, axis=0).T)
    # most steps are inside a polyline; jumps between polylines are longer
    assert np.median(d) == pytest.approx(I.SPACING, abs=1e-4)


def test_dense_headway_and_rain():
    """The 32-vehicle intersections spawn at 6-10 m headway, with rain films."""
    w = I.intersections(8, 32, seed=3, headway=(6.0, 10.0), rain=True)
    check_worlds(w)
    assert np.all(np.diff(w.agent_offsets) == 32)
    assert np.all((w.film_mm >= 0.0) & (w.film_mm <= 0.8))
    for k in range(w.num_worlds):
        s = w.spawn[w.spawn_offsets[k]:w.spawn_offsets[k] + 32]
        dx = s[None, :, 0] - s[:, None, 0]
        dy = s[None, :, 1] - s[:, None, 1]
        d = np.hypot(dx, dy)
        np.fill_diagonal(d, np.inf)
        # neighbouring lanes are a lane width apart
        assert d.min() >= I.LANE_W - 0.1
        # along one lane (same heading, no lateral offset) the gap is the headway
        hx, hy = np.cos(s[:, 2]), np.sin(s[:, 2])
        lateral = np.abs(hx[:, None] * dy - hy[:, None] * dx)
        same = (lateral < 0.5) & (np.cos(s[:, None, 2] - s[None, :, 2]) > 0.99)
        assert np.all(d[same] >= 5.9)


@pytest.mark.parametrize("name", ["plane1x2", "cross64x8", "uneven256"])
def test_seed_determinism(name):
    a, b, c = I.workload(name, seed=0), I.workload(name, seed=0), I.workload(name, seed=1)
    for f in ("agent_offsets", "road_xy", "tri_verts", "spawn", "mu_class"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    if name != "plane1x2":
        assert not np.array_equal(a.spawn, c.spawn)


def test_actions_and_policy_params_are_seeded():
    assert np.array_equal(I.actions(3, 7, 100), I.actions(3, 7, 100))
    assert not np.array_equal(I.actions(3, 7, 100), I.actions(3, 8, 100))
    x = I.actions(1, 2, 10000)
    assert np.all(np.abs(x[:, 0]) <= 1.0) and np.all(np.abs(x[:, 1]) <= 0.5)
    Ws, bs = I.mlp_params([256, 256, 256, 2], seed=0)
    assert [W.shape for W in Ws] == [(256, 256), (256, 256), (2, 256)]
    assert all(np.all(b == 0) for b in bs)
    assert abs(Ws[0].std() - 1 / 16) < 0.005
