"""FP64 reference of the on-device PPO update -- test infrastructure only
(tests, the smoke check and bench.py's CPU baseline may use it; the product
path never does).

What it computes (Algorithm "SceneFactory Pipeline", the PPO update after T
rollout steps; appendix "PPO Hyperparameters", Table "PPO hyperparameters";
appendix "Network Architecture Details" for the network):

* the late-fusion actor-critic forward pass of ``oracle.actor_critic`` in
  float64 torch tensors, with the same bf16 rounding points (inputs, weights,
  hidden activations) taken straight through for the gradient: a rounded
  value is used in the products, its derivative is that of the unrounded
  one;
* a diagonal Gaussian policy over the 3-dim action (throttle, steering,
  brake) with the actor's mean and its state-independent log sigma;
* generalised advantage estimation (Schulman et al. 2016) over the rollout,
  a terminal step cutting both the bootstrap and the recursion;
* the clipped surrogate objective (Schulman et al. 2017), the squared value
  error and the Gaussian entropy, combined as
  ``surrogate + c_v * value_loss - c_e * entropy``;
* the mean KL divergence between the rollout's policy and the current one,
  which halves or doubles the learning rate around its target;
* gradient clipping to a global norm and Adam (Kingma and Ba 2015).

Readings where the paper is silent are listed in the design notes; the
gradient itself comes from torch autograd (a library primitive) over these
definitions.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from oracle import oracle as O

EGO, RK, VK = O.FULL_EGO, O.FULL_ROAD_K, O.FULL_NEIGH_K
LOG_2PI = math.log(2.0 * math.pi)


ROUND = [True]       # bf16 rounding points on (switched off only by pins)


def bf16r(x: np.ndarray) -> np.ndarray:
    """Round float64 values to 8 significant bits, ties to even (bf16)."""
    x = np.asarray(x, np.float64)
    if not ROUND[0]:
        return x
    m, e = np.frexp(x)
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)


def _st(t: torch.Tensor) -> torch.Tensor:
    """bf16-rounded value, gradient of the unrounded one (straight through)."""
    r = torch.from_numpy(bf16r(t.detach().numpy()))
    return t + (r - t).detach()


def _elu(z: torch.Tensor) -> torch.Tensor:
    return torch.where(z > 0, z, torch.expm1(torch.clamp(z, max=0.0)))


def _dense(P: torch.Tensor, off: int, n_in: int, n_out: int, x: torch.Tensor, act: bool):
    W = P[off:off + n_in * n_out].reshape(n_out, n_in)
    b = P[off + n_in * n_out:off + n_in * n_out + n_out]
    z = x @ _st(W).T + b
    return (_st(_elu(z)) if act else z), off + n_in * n_out + n_out


def _first_max(z: torch.Tensor) -> torch.Tensor:
    """Index of the first maximum along dim 0 (a tie keeps the lower slot)."""
    zd = z.detach()
    top = zd.max(dim=0, keepdim=True).values
    hit = (zd == top).to(torch.int64)
    first = hit * (torch.cumsum(hit, dim=0) == 1).to(torch.int64)
    return first.argmax(dim=0)


def _encoder_pool(P, off, n_in, x: torch.Tensor):
    """Set encoder n_in -> 96 -> 96 on the valid rows of x, masked max-pool
    (an empty set pools to 0)."""
    end = off + n_in * 96 + 96 + 96 * 96 + 96
    if x.shape[0] == 0:
        return torch.zeros(96, dtype=torch.float64), end
    h, o2 = _dense(P, off, n_in, 96, _st(x), True)
    z, _ = _dense(P, o2, 96, 96, h, True)
    idx = _first_max(z)
    return z.gather(0, idx[None, :])[0], end


def _net(P: torch.Tensor, off: int, o: torch.Tensor, nr: int, nv: int, nout: int):
    e1, off = _dense(P, off, EGO, 64, _st(o[:EGO]), True)
    e2, off = _dense(P, off, 64, 64, e1, True)
    road = o[EGO:EGO + 5 * RK].reshape(RK, 5)[:nr]
    veh = o[EGO + 5 * RK:].reshape(VK, 7)[:nv]
    pr, off = _encoder_pool(P, off, 5, road)
    pv, off = _encoder_pool(P, off, 7, veh)
    emb = torch.cat([e2, pr, pv])
    t1, off = _dense(P, off, 256, 128, emb, True)
    t2, off = _dense(P, off, 128, 64, t1, True)
    out, off = _dense(P, off, 64, nout, t2, False)
    return out, off


def forward(P: torch.Tensor, obs: np.ndarray, counts: np.ndarray):
    """Mean [M, 3] and value [M] of the actor-critic (float64 tensors that
    carry the graph to P, a float64 tensor of the float32 parameters)."""
    obs_t = torch.from_numpy(np.ascontiguousarray(obs, np.float32).astype(np.float64))
    means, values = [], []
    for r in range(obs_t.shape[0]):
        nr, nv = int(counts[r, 0]), int(counts[r, 1])
        m, off = _net(P, 0, obs_t[r], min(nr, RK), min(nv, VK), 3)
        off += 3                                   # log sigma
        v, _ = _net(P, off, obs_t[r], min(nr, RK), min(nv, VK), 1)
        means.append(m)
        values.append(v[0])
    return torch.stack(means), torch.stack(values)


def log_std_slice() -> slice:
    a = O.AC_BODY + 3 * 64 + 3
    return slice(a, a + 3)


def gaussian_logp(u, mean, log_std):
    """log N(u; mean, diag exp(2 log_std)) summed over the 3 action dims."""
    return (-0.5 * ((u - mean) / torch.exp(log_std)) ** 2 - log_std - 0.5 * LOG_2PI).sum(-1)


def gaussian_entropy(log_std):
    return (log_std + 0.5 * (1.0 + LOG_2PI)).sum()


def gaussian_kl(mu0, ls0, mu1, ls1):
    """KL(N(mu0, s0^2) || N(mu1, s1^2)) summed over the action dims."""
    return (ls1 - ls0 + (torch.exp(2 * ls0) + (mu0 - mu1) ** 2) / (2 * torch.exp(2 * ls1)) - 0.5).sum(-1)


def gae(rewards, dones, values, last_value, gamma, lam):
    """Advantages and returns over a rollout [T][N]: delta_t = r_t +
    gamma V_{t+1} (1 - d_t) - V_t, A_t = delta_t + gamma lam (1 - d_t) A_{t+1},
    R_t = A_t + V_t, with V_T the bootstrap value of the state after the
    last step."""
    r = np.asarray(rewards, np.float64)
    d = np.asarray(dones, np.float64)
    v = np.asarray(values, np.float64)
    T = r.shape[0]
    adv = np.zeros_like(r)
    nxt_v = np.asarray(last_value, np.float64)
    nxt_a = np.zeros(r.shape[1])
    for t in range(T - 1, -1, -1):
        delta = r[t] + gamma * nxt_v * (1.0 - d[t]) - v[t]
        nxt_a = delta + gamma * lam * (1.0 - d[t]) * nxt_a
        adv[t] = nxt_a
        nxt_v = v[t]
    return adv, adv + v


def normalise(adv):
    """Advantages less their mean over the batch, over their standard
    deviation (population, plus 1e-8)."""
    a = np.asarray(adv, np.float64)
    return (a - a.mean()) / (a.std() + 1e-8)


def loss_and_grad(params, obs, counts, u, logp_old, mu_old, log_std_old, adv, ret, clip, c_v, c_e):
    """PPO loss of one minibatch and its gradient over the parameter block.
    Returns (loss, grad float64 [AC_PARAMS], stats dict)."""
    P = torch.tensor(np.asarray(params, np.float32).astype(np.float64), requires_grad=True)
    mean, value = forward(P, obs, counts)
    ls = P[log_std_slice()]
    u_t = torch.from_numpy(np.asarray(u, np.float64))
    lp = gaussian_logp(u_t, mean, ls)
    ratio = torch.exp(lp - torch.from_numpy(np.asarray(logp_old, np.float64)))
    A = torch.from_numpy(np.asarray(adv, np.float64))
    surr = torch.maximum(-A * ratio, -A * torch.clamp(ratio, 1.0 - clip, 1.0 + clip)).mean()
    vloss = ((value - torch.from_numpy(np.asarray(ret, np.float64))) ** 2).mean()
    ent = gaussian_entropy(ls)
    loss = surr + c_v * vloss - c_e * ent
    loss.backward()
    with torch.no_grad():
        kl = gaussian_kl(torch.from_numpy(np.asarray(mu_old, np.float64)),
                         torch.from_numpy(np.asarray(log_std_old, np.float64)), mean, ls).mean()
        clipped = ((ratio - 1.0).abs() > clip).to(torch.float64).mean()
    stats = {"surrogate": surr.item(), "value_loss": vloss.item(), "entropy": ent.item(), "kl": kl.item(),
             "clip_fraction": clipped.item(), "mean": mean.detach().numpy(), "value": value.detach().numpy()}
    return loss.item(), P.grad.numpy().copy(), stats


def adapt_lr(lr, kl, target, lr_min, lr_max):
    """Halve the rate above twice the KL target, double it below half."""
    if kl > 2.0 * target:
        return max(lr_min, lr / 2.0)
    if kl < 0.5 * target:
        return min(lr_max, lr * 2.0)
    return lr


def clip_grad(g, max_norm):
    n = float(np.sqrt(np.sum(np.asarray(g, np.float64) ** 2)))
    return np.asarray(g, np.float64) * min(1.0, max_norm / (n + 1e-6)), n
