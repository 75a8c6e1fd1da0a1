"""Pins of the PPO reference (oracle/ppo.py) against what the mathematics
fixes: the network against the C oracle's forward pass, autograd against
central finite differences, GAE against its closed forms (lambda = 1: the
discounted return to go less V; lambda = 0: the one-step TD error) and a
hand-worked rollout with a terminal step, the Gaussian log-density,
entropy and KL against scipy, the clipped objective's dead zones, and the
learning-rate rule."""
import math

import numpy as np
import pytest

scipy_stats = pytest.importorskip("scipy.stats")
from scipy import integrate

from oracle import oracle as O
from oracle import ppo

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def built():
    O.build()


def small_batch(seed, M=5, nr=(0, 7, 350, 3, 12), nv=(2, 0, 24, 5, 1)):
    rng = np.random.default_rng(seed)
    obs = rng.uniform(-1.0, 1.0, (M, O.FULL_DIM)).astype(np.float32)
    counts = np.array(list(zip(nr, nv)), np.int32)[:M]
    P = (rng.standard_normal(O.AC_PARAMS) * 0.15).astype(np.float32)
    return obs, counts, P


def test_forward_matches_the_c_oracle():
    obs, counts, P = small_batch(1)
    mean_c, value_c = O.actor_critic(P, obs, counts)
    mean_t, value_t = ppo.forward(torch.tensor(P.astype(np.float64)), obs, counts)
    assert np.allclose(mean_t.detach().numpy(), mean_c, rtol=0, atol=1e-12)
    assert np.allclose(value_t.detach().numpy(), value_c, rtol=0, atol=1e-12)


def test_gradient_matches_finite_differences():
    """Rounding off: the loss's autograd gradient against central
    differences on parameters of every part (ego, road and vehicle encoders,
    trunk, both heads, log sigma), away from max-pool ties."""
    obs, counts, P = small_batch(2, M=3, nr=(9, 4, 0), nv=(3, 0, 2))
    rng = np.random.default_rng(3)
    u = rng.standard_normal((3, 3))
    adv = np.array([0.7, -1.2, 0.4])
    ret = np.array([0.3, -0.5, 1.1])
    ppo.ROUND[0] = False
    try:
        P64 = P.astype(np.float64)
        mean0, _ = ppo.forward(torch.tensor(P64), obs, counts)
        ls0 = P64[ppo.log_std_slice()]
        logp_old = ppo.gaussian_logp(torch.tensor(u), mean0, torch.tensor(ls0)).numpy() + 0.05
        args = (obs, counts, u, logp_old, mean0.detach().numpy(), ls0, adv, ret, 0.15, 1.0, 3e-5)

        def loss_at(p64):
            Pt = torch.tensor(p64)
            m, v = ppo.forward(Pt, obs, counts)
            ls = Pt[ppo.log_std_slice()]
            ratio = torch.exp(ppo.gaussian_logp(torch.tensor(u), m, ls) - torch.tensor(logp_old))
            A = torch.tensor(adv)
            surr = torch.maximum(-A * ratio, -A * torch.clamp(ratio, 0.85, 1.15)).mean()
            return float(surr + ((v - torch.tensor(ret)) ** 2).mean() - 3e-5 * ppo.gaussian_entropy(ls))

        # the oracle's gradient is taken at float32 parameters: use them exactly
        _, g, _ = ppo.loss_and_grad(P, *args)
        body = O.AC_BODY
        picks = [0, 11 * 64 + 3, 64 * 12 + 64 * 64 + 7, 64 * 12 + 64 * 64 + 5 * 96 + 96 + 200,
                 body - 64 * 128 - 64 - 5, body + 10, body + 3 * 64 + 1, body + 3 * 64 + 3,
                 body + 3 * 64 + 5, body + 3 * 64 + 6 + 300, O.AC_PARAMS - 2, O.AC_PARAMS - 1]
        for k in picks:
            h = 1e-5 * max(1.0, abs(P64[k]))
            pp, pm = P64.copy(), P64.copy()
            pp[k] += h
            pm[k] -= h
            fd = (loss_at(pp) - loss_at(pm)) / (2 * h)
            assert abs(g[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, g[k], fd)
    finally:
        ppo.ROUND[0] = True


def test_gae_closed_forms_and_a_terminal_step():
    rng = np.random.default_rng(4)
    T, N, g = 6, 3, 0.9
    r = rng.standard_normal((T, N))
    v = rng.standard_normal((T, N))
    last = rng.standard_normal(N)
    d = np.zeros((T, N))
    # lambda = 1: discounted return to go (bootstrapped) less V
    adv, ret = ppo.gae(r, d, v, last, g, 1.0)
    want = np.array([[sum(g ** (k - t) * r[k, n] for k in range(t, T)) + g ** (T - t) * last[n]
                      for n in range(N)] for t in range(T)])
    assert np.allclose(ret, want, atol=1e-12) and np.allclose(adv, want - v, atol=1e-12)
    # lambda = 0: the one-step TD error
    adv0, _ = ppo.gae(r, d, v, last, g, 0.0)
    nxt = np.vstack([v[1:], last[None]])
    assert np.allclose(adv0, r + g * nxt - v, atol=1e-12)
    # a terminal step at t = 2 of agent 0 (hand-worked, gamma 0.5, lambda 0.5)
    r2 = np.array([[1.0], [2.0], [3.0], [4.0]])
    v2 = np.array([[0.5], [0.25], [1.0], [2.0]])
    d2 = np.array([[0.0], [0.0], [1.0], [0.0]])
    a2, _ = ppo.gae(r2, d2, v2, np.array([8.0]), 0.5, 0.5)
    d3 = 4.0 + 0.5 * 8.0 - 2.0           # 6
    dd2 = 3.0 - 1.0                      # terminal: no bootstrap, 2
    dd1 = 2.0 + 0.5 * 1.0 - 0.25         # 2.25
    dd0 = 1.0 + 0.5 * 0.25 - 0.5         # 0.625
    a = [dd0 + 0.25 * (dd1 + 0.25 * dd2), dd1 + 0.25 * dd2, dd2, d3]
    assert np.allclose(a2[:, 0], a, atol=1e-12)


def test_gaussian_logp_entropy_kl_against_scipy():
    rng = np.random.default_rng(5)
    mu, ls, u = rng.standard_normal(3), rng.standard_normal(3) * 0.3, rng.standard_normal(3)
    lp = float(ppo.gaussian_logp(torch.tensor(u), torch.tensor(mu), torch.tensor(ls)))
    assert abs(lp - scipy_stats.norm.logpdf(u, mu, np.exp(ls)).sum()) < 1e-12
    ent = float(ppo.gaussian_entropy(torch.tensor(ls)))
    assert abs(ent - scipy_stats.norm(mu, np.exp(ls)).entropy().sum()) < 1e-12
    mu1, ls1 = mu + 0.3, ls - 0.2
    kl = float(ppo.gaussian_kl(torch.tensor(mu), torch.tensor(ls), torch.tensor(mu1), torch.tensor(ls1)))
    num = 0.0
    for k in range(3):
        p = scipy_stats.norm(mu[k], np.exp(ls[k]))
        q = scipy_stats.norm(mu1[k], np.exp(ls1[k]))
        num += integrate.quad(lambda x: p.pdf(x) * (p.logpdf(x) - q.logpdf(x)), -30, 30, limit=200)[0]
    assert abs(kl - num) < 1e-8


def test_clipped_objective_dead_zones():
    """A > 0 with the ratio above 1 + eps, or A < 0 below 1 - eps: the
    surrogate passes no gradient to the mean; inside the band it is
    -A * ratio * d log p."""
    mu = torch.zeros(1, 3, dtype=torch.float64, requires_grad=True)
    ls = torch.zeros(3, dtype=torch.float64)
    u = torch.tensor([[0.5, -0.2, 0.1]], dtype=torch.float64)
    lp0 = float(ppo.gaussian_logp(u, torch.zeros(1, 3, dtype=torch.float64), ls))
    for A, shift, dead in ((1.0, 0.5, True), (-1.0, -0.5, True), (1.0, 0.05, False), (-1.0, 0.05, False)):
        mu.grad = None
        lp_old = lp0 - shift                     # ratio = exp(shift) at mu = 0
        ratio = torch.exp(ppo.gaussian_logp(u, mu, ls) - lp_old)
        At = torch.tensor([A], dtype=torch.float64)
        surr = torch.maximum(-At * ratio, -At * torch.clamp(ratio, 0.85, 1.15)).mean()
        surr.backward()
        if dead:
            assert torch.all(mu.grad == 0)
        else:
            want = -A * math.exp(shift) * (u[0] - 0.0)   # d log p / d mu = (u - mu) / sigma^2
            assert torch.allclose(mu.grad[0], want, atol=1e-12)


def test_learning_rate_rule():
    assert ppo.adapt_lr(1e-3, 0.03, 0.01, 1e-5, 1e-2) == 5e-4
    assert ppo.adapt_lr(1e-3, 0.004, 0.01, 1e-5, 1e-2) == 2e-3
    assert ppo.adapt_lr(1e-3, 0.01, 0.01, 1e-5, 1e-2) == 1e-3
    assert ppo.adapt_lr(1.5e-5, 0.5, 0.01, 1e-5, 1e-2) == 1e-5
    assert ppo.adapt_lr(8e-3, 0.0, 0.01, 1e-5, 1e-2) == 1e-2
    g, n = ppo.clip_grad(np.array([3.0, 4.0]), 1.0)
    assert abs(n - 5.0) < 1e-12 and np.allclose(g, [0.6, 0.8], atol=1e-6)
