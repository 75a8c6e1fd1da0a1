"""The learned tire surrogate through the C ABI against the FP64 oracle.

* sample log: the training samples the step writes (inputs and the plain
  tire model's outputs) match the oracle's for the same state;
* training kernels: the full-batch gradient of the mean squared error and
  the Adam update match the oracle's gradient and Adam;
* inference: the batched predictions match the oracle's forward pass with
  the same bf16 rounding points;
* accuracy: trained on logged samples, the network reaches a mean relative
  force error of at most 2 % on samples of a different run;
* in-step use: with a trained network both sides take the same wheel
  decisions (up to rare threshold cases) and the same states; a network
  whose predictions fail the residual checks, or an empty envelope, leaves
  the step bit-identical to the plain step.
"""
import numpy as np
import pytest

from paper_2605_08528_amd import inputs as I
from tests.helpers import params as mkparams

pytestmark = pytest.mark.gpu

SIZES = [16, 128, 128, 128, 3]


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


def layers(flat):
    """Parameter block -> ([W1..W4], [b1..b4]) with W as [out, in]."""
    Ws, bs, o = [], [], 0
    for a, b in zip(SIZES[:-1], SIZES[1:]):
        Ws.append(flat[o:o + a * b].reshape(b, a))
        o += a * b
        bs.append(flat[o:o + b])
        o += b
    assert o == flat.size
    return Ws, bs


def moving(speed_lo=5.0, speed_hi=14.0, seed=0):
    """init callback: every agent moving forward along its heading, wheels
    rolling without slip"""
    def init(f, k):
        rng = np.random.default_rng(seed)
        n = f.shape[1]
        spd = rng.uniform(speed_lo, speed_hi, n).astype(np.float32)
        qw, qz = f[3], f[6]
        yaw = 2.0 * np.arctan2(qz, qw)
        f[7] = spd * np.cos(yaw)
        f[8] = spd * np.sin(yaw)
        for c in range(4):
            f[13 + c] = spd / 0.35
    return init


def make(O, torch, worlds, flags=0, init=None):
    from paper_2605_08528_amd import sf
    p = mkparams()
    sim = sf.Sim(worlds, p, flags=flags)
    if init is not None:
        f, k = sim.get_state()
        init(f, k)
        sim.set_state(f, k)
    orc = O.Oracle(worlds, p, invincible=bool(flags & sf.SF_INVINCIBLE))
    return sim, orc


def cuda(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gather_samples(torch, worlds, steps, seed, capacity=1 << 20):
    """Run the plain step with random actions and return the valid logged
    samples as a device tensor."""
    from paper_2605_08528_amd import sf
    sim = sf.Sim(worlds, mkparams(), flags=sf.SF_INVINCIBLE | sf.SF_AUTO_RESET)
    f, k = sim.get_state()
    moving(seed=seed)(f, k)
    sim.set_state(f, k)
    dt, S = 1.0 / 30.0, 4
    sim.sur_log(capacity)
    for step in range(steps):
        a = I.actions(seed, step, sim.N)
        a[:, 0] = 0.6 * a[:, 0] + 0.2   # mostly driving on
        sim.step(cuda(torch, a), dt, S)
    data, n = sim.sur_collect(capacity)
    torch.cuda.synchronize()
    return sim, data.clone()


# ---------------------------------------------------------- sample log
def test_sample_log_matches_oracle(O, torch):
    w = I.intersections(8, 8, seed=4)
    sim, orc = make(O, torch, w, flags=1, init=moving(seed=1))
    N = sim.N
    dt = float(np.float32(1.0 / 30.0))
    sim.sur_log(4 * N)          # one substep per step: the ring holds one step
    orc.record_samples(True)
    worst_f = worst_t = 0.0
    n_valid = 0
    for step in range(12):
        f, k = sim.get_state()
        orc.set_state(f.astype(np.float64), k)
        a = I.actions(7, step, N)
        a[:, 0] = 0.5 * np.abs(a[:, 0])
        sim.step(cuda(torch, a), dt, 1)
        orc.step(a, dt, 1)
        ref = orc.samples().reshape(N * 4, 20)
        got, n = sim.sur_collect(4 * N)
        got = got.cpu().numpy()
        valid = ref[:, 19] == 1.0
        assert n == int(valid.sum()), (step, n, int(valid.sum()))
        r = ref[valid]
        worst_f = max(worst_f, float(np.abs(got[:, :16] - r[:, :16]).max(initial=0)))
        worst_t = max(worst_t, float(np.abs(got[:, 16:19] - r[:, 16:19]).max(initial=0)))
        n_valid += n
    print(f"sample log: {n_valid} samples, worst input diff {worst_f:.3g}, target diff {worst_t:.3g}")
    assert n_valid > 100
    assert worst_f <= 1e-4 and worst_t <= 1e-4
    sim.close()


# ----------------------------------------------------- training kernels
def random_data(M, seed):
    rng = np.random.default_rng(seed)
    d = np.zeros((M, 20), np.float32)
    d[:, :16] = rng.uniform(-1.0, 1.0, (M, 16))
    d[:, 16:19] = rng.uniform(-1.0, 1.0, (M, 3))
    d[:, 19] = 1.0
    return d


def fresh_sim(torch):
    from paper_2605_08528_amd import sf
    return sf.Sim(I.workload("plane1x2"), mkparams())


def test_gradient_matches_oracle(O, torch):
    sim = fresh_sim(torch)
    M = 1000                      # 15 full tiles and a ragged one of 40
    d = random_data(M, 3)
    dd = cuda(torch, d)
    sim.sur_train(dd, steps=0, init_seed=11, set_envelope=True)
    P0, lo, hi = sim.sur_get()
    assert np.array_equal(lo, d[:, :16].min(0)) and np.array_equal(hi, d[:, :16].max(0))
    loss_g, g = sim.sur_gradient(dd)
    Ws, bs = layers(P0)
    loss_o, gW, gb = O.mlp_mse_grad(Ws, bs, d[:, :16], d[:, 16:19], row_weight=O.force_weights(d[:, 16:19]))
    assert abs(loss_g - loss_o) <= 1e-4 * loss_o, (loss_g, loss_o)
    gWg, gbg = layers(g.astype(np.float64))
    for l in range(4):
        for a, b in ((gWg[l], gW[l]), (gbg[l], gb[l])):
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            mx = np.abs(a - b).max() / np.abs(b).max()
            print("layer", l, "gradient relative norm error", rel, "max abs / max", mx)
            assert rel <= 1e-2, (l, rel)
            # every entry: within 2 % of the tensor's largest gradient
            assert mx <= 2e-2, (l, mx)
    sim.close()


def test_adam_steps_match_oracle(O, torch):
    sim = fresh_sim(torch)
    d = random_data(700, 5)
    dd = cuda(torch, d)
    sim.sur_train(dd, steps=0, init_seed=3)
    w, _, _ = sim.sur_get()
    m = np.zeros(w.size, np.float64)
    v = np.zeros(w.size, np.float64)
    for t in (1, 2, 3):
        _, g = sim.sur_gradient(dd)        # the gradient the GPU step uses
        sim.sur_train(dd, steps=1, batch=0, lr=1e-3)
        O.adam(w, g, m, v, t, 1e-3)
        got, _, _ = sim.sur_get()
        assert np.allclose(got, w, rtol=1e-6, atol=1e-7), (t, float(np.abs(got - w).max()))
        w = got.copy()                     # continue from the GPU's rounding
    sim.close()


def test_predict_matches_oracle(O, torch):
    sim = fresh_sim(torch)
    d = random_data(333, 9)
    dd = cuda(torch, d)
    sim.sur_train(dd, steps=20, batch=0, lr=1e-3, init_seed=5)
    P, _, _ = sim.sur_get()
    y = sim.sur_predict(dd).cpu().numpy()
    Ws, bs = layers(P)
    O.set_bf16(True)
    yo = O.mlp_forward(Ws, bs, d[:, :16])
    err = np.abs(y - yo).max()
    scale = max(1.0, float(np.abs(yo).max()))
    rel = np.linalg.norm(y - yo) / np.linalg.norm(yo)
    print(f"predict: worst |gpu - oracle| {err:.3g} over outputs of scale {scale:.3g}, relative norm {rel:.3g}, "
          f"{int(np.sum(np.abs(y - yo) > 1e-3 * scale))} of {y.size} outputs beyond 1e-3")
    # both sides round inputs, weights and hidden activations to bf16 at the
    # same points; a hidden value that lands on a rounding boundary under the
    # fp32 (GPU) or fp64 (oracle) sum flips by one bf16 ulp (2^-8 relative),
    # which moves an output by up to a few 2^-8 of its scale
    assert rel <= 1e-3
    assert err <= 4e-3 * scale
    sim.close()


def test_errors_per_sample(torch):
    """Per-sample relative force errors equal |d(F_x, F_y)| / max(|(F_x, F_y)|,
    0.05) of the network's predictions against the stored targets (both in
    units of mu F_z), and their mean is the evaluation's mean."""
    sim = fresh_sim(torch)
    d = random_data(777, 13)
    dd = cuda(torch, d)
    sim.sur_train(dd, steps=20, batch=0, lr=1e-3, init_seed=5)
    y = sim.sur_predict(dd).cpu().numpy().astype(np.float64)
    e = sim.sur_errors(dd).cpu().numpy().astype(np.float64)
    t = d[:, 16:18].astype(np.float64)
    ref = np.hypot(y[:, 0] - t[:, 0], y[:, 1] - t[:, 1]) / np.maximum(np.hypot(t[:, 0], t[:, 1]), 0.05)
    assert e.shape == (777,)
    assert np.allclose(e, ref, rtol=1e-5, atol=1e-6)
    m, p95 = sim.sur_evaluate(dd)
    assert abs(m - e.mean()) <= 1e-5 * max(1.0, m)
    assert np.sum(e <= p95) >= 0.95 * len(e)
    sim.close()


# ------------------------------------------------------------ accuracy
@pytest.fixture(scope="module")
def trained(torch):
    """A network trained on samples of one run; held-out samples of another."""
    w_train = I.intersections(32, 16, seed=21)
    w_test = I.intersections(16, 16, seed=22)
    s1, train = gather_samples(torch, w_train, 60, seed=1)
    s2, test = gather_samples(torch, w_test, 30, seed=2)
    s1.sur_train(train, steps=0, init_seed=1, set_envelope=True)
    before = s1.sur_evaluate(test)
    loss = s1.sur_fit(train)
    after = s1.sur_evaluate(test)
    P, lo, hi = s1.sur_get()
    s2.close()
    s1.close()
    print(f"surrogate: {train.shape[0]} training / {test.shape[0]} test samples; "
          f"mean rel force error untrained {before[0]:.4f}, trained {after[0]:.4f} "
          f"(p95 {after[1]:.4f}), last loss {loss:.3g}")
    return {"P": P, "lo": lo, "hi": hi, "before": before, "after": after, "n": train.shape[0]}


def test_training_reaches_two_percent(trained):
    assert trained["n"] > 50000
    assert trained["after"][0] <= 0.02
    assert trained["after"][0] < 0.25 * trained["before"][0]


# ------------------------------------------------------- in-step use
GROUPS = {"p": ([0, 1, 2], 1.0), "q": ([3, 4, 5, 6], 1.0), "v": ([7, 8, 9], 1.0),
          "w": ([10, 11, 12], 1.0), "om": ([13, 14, 15, 16], 1.0), "th": ([17], 0.01),
          "thd": ([18], 1.0)}


def group_err(fg, fo):
    out = {}
    for g, (rows, s) in GROUPS.items():
        e = np.abs(fg[rows].astype(np.float64) - fo[rows]) / np.maximum(np.abs(fo[rows]), s)
        out[g] = e.max(axis=0)
    return out


def test_surrogate_step_lockstep(O, torch, trained):
    """Both sides use the trained network inside the step.  A wheel whose
    input or prediction sits on a threshold (envelope bound, friction circle,
    slip sign) can take the other branch on the other side; such cases are
    rare and counted, every other agent matches within 2e-3."""
    w = I.intersections(16, 8, seed=6)
    sim, orc = make(O, torch, w, flags=1, init=moving(seed=3))
    N = sim.N
    sim.sur_set(trained["P"], trained["lo"], trained["hi"])
    sim.sur_enable(True)
    orc.set_surrogate(trained["P"], trained["lo"], trained["hi"], True)
    dt = float(np.float32(1.0 / 30.0))
    worst = {g: 0.0 for g in GROUPS}
    off = 0
    for step in range(20):
        f, k = sim.get_state()
        orc.set_state(f.astype(np.float64), k)
        a = I.actions(5, step, N)
        a[:, 0] = 0.5 * np.abs(a[:, 0])
        sim.step(cuda(torch, a), dt, 4)
        orc.step(a, dt, 4)
        fg, kg = sim.get_state()
        fo, ko = orc.get_state()
        assert np.array_equal(kg, ko), step
        e = group_err(fg, fo)
        bad = np.zeros(N, bool)
        for g in GROUPS:
            bad |= e[g] > 2e-3
        off += int(bad.sum())
        for g in GROUPS:
            worst[g] = max(worst[g], float(e[g][~bad].max(initial=0)))
    used_g, fb_g = sim.sur_counts()
    used_o, fb_o = orc.surrogate_counts()
    print(f"surrogate lockstep: gpu used/fallback {used_g}/{fb_g}, oracle {used_o}/{fb_o}; "
          f"agent-steps off {off} of {20 * N}; worst {worst}")
    assert used_o > 0.5 * (used_o + fb_o)
    assert abs(used_g - used_o) <= max(4, 0.002 * used_o)
    # the domain test (F_z > 0, |v_x| >= 3 m/s) of a later substep can flip
    # for a wheel on the threshold, since the substeps after the first start
    # from float states that differ in the last bits
    assert abs((used_g + fb_g) - (used_o + fb_o)) <= max(8, 0.001 * (used_o + fb_o))
    assert off <= max(2, 0.005 * 20 * N)
    sim.close()


def plain_states(torch, w, steps, setup=None):
    from paper_2605_08528_amd import sf
    sim = sf.Sim(w, mkparams(), flags=1)
    f, k = sim.get_state()
    moving(seed=4)(f, k)
    sim.set_state(f, k)
    if setup:
        setup(sim)
    out = []
    for step in range(steps):
        a = I.actions(8, step, sim.N)
        sim.step(cuda(torch, a), 1.0 / 30.0, 4)
        out.append(sim.get_state()[0])
    counts = sim.sur_counts() if setup else None
    sim.close()
    return out, counts


def test_fallback_is_the_plain_step(torch, trained):
    """An empty envelope, or a network that always fails the friction-circle
    check, leaves every wheel on the plain model: states bit-identical."""
    w = I.intersections(8, 8, seed=12)
    ref, _ = plain_states(torch, w, 15)
    P = trained["P"]

    def empty(sim):
        sim.sur_set(P, trained["hi"] + 1.0, trained["hi"] + 2.0)
        sim.sur_enable(True)

    bad = P.copy()
    bad[-3:] = [10.0, 10.0, 0.0]       # outputs far outside the friction circle

    def outside(sim):
        sim.sur_set(bad, np.full(16, -1e30, np.float32), np.full(16, 1e30, np.float32))
        sim.sur_enable(True)

    for setup in (empty, outside):
        got, (used, fb) = plain_states(torch, w, 15, setup)
        assert used == 0 and fb > 0
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


def test_cross1024x16_surrogate_full_size_sampled(O, torch):
    """The learned-tire step at full size (1024 worlds x 16 vehicles, the
    configuration the network is meant for): a network trained on samples of
    this workload, then sampled worlds re-run on the oracle with the same
    network from the GPU state."""
    from paper_2605_08528_amd import sf
    from tests.test_gpu_parity import sampled_full_size
    w = I.workload("cross1024x16")
    sim = sf.Sim(w, mkparams(), flags=sf.SF_AUTO_RESET)
    f, k = sim.get_state()
    moving(seed=9)(f, k)
    sim.set_state(f, k)
    sim.sur_log(1 << 22)
    for step in range(12):
        a = I.actions(13, step, sim.N)
        a[:, 0] = 0.5 * a[:, 0] + 0.3
        sim.step(cuda(torch, a), 1.0 / 60.0, 4)
    data, n = sim.sur_collect(1 << 22)
    sim.sur_fit(data[: min(n, 1 << 22)])
    P, lo, hi = sim.sur_get()
    sim.close()
    sampled_full_size(O, torch, "cross1024x16", {"step_grid": 512}, n_sample=4, surrogate=(P, lo, hi),
                      init=moving(seed=10))


def test_captured_graph_dropped_by_surrogate_changes(torch):
    """A captured graph holds the sample ring, the envelope and the step
    variant as kernel arguments: logging on or off, switching the network
    on or off, loading parameters and training with a new envelope each drop
    it, so a replay can never write into a freed ring or run a stale
    envelope (sf_graph_launch then reports that no graph is captured)."""
    from paper_2605_08528_amd import sf
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim = sf.Sim(I.intersections(2, 4, seed=3), mkparams(), flags=sf.SF_AUTO_RESET, stream=stream)
        sim.policy_load(*I.mlp_params([256, 256, 256, 2], seed=1))
        d = cuda(torch, random_data(256, 5))
        sim.sur_train(d, steps=0, init_seed=3, set_envelope=True)
        P, lo, hi = sim.sur_get()
        changes = [("log on", lambda: sim.sur_log(4096)), ("log off", lambda: sim.sur_log(0)),
                   ("network on", lambda: sim.sur_enable(True)), ("network off", lambda: sim.sur_enable(False)),
                   ("set", lambda: sim.sur_set(P, lo, hi)),
                   ("train with envelope", lambda: sim.sur_train(d, steps=1, set_envelope=True))]
        for name, change in changes:
            sim.graph_capture(2, 1.0 / 30.0, 4)
            sim.graph_launch()
            change()
            with pytest.raises(sf.SFError, match="no graph captured"):
                sim.graph_launch()
        # training without a new envelope keeps the graph (weights are read
        # from device memory by every replay)
        sim.graph_capture(2, 1.0 / 30.0, 4)
        sim.sur_train(d, steps=1)
        sim.graph_launch()
        torch.cuda.synchronize()
        sim.close()
