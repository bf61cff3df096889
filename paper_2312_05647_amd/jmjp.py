"""The jump-based method J-MJP (Method #2, Sec. 2.2.2, Eq. sample_J-MJP):
a Gibbs sampler over the log-rates psi = log(theta) and the latent numbers
of virtual jumps k^i of every observation, batched over chains.

* k | s, theta (Eq. sam_k): each k^i separately, proposal
  Poisson(Omega_theta T^i) (the SI's choice, equal to its prior), accepted
  with min(1, p(s^i | k'^i, theta) / p(s^i | k^i, theta)).
* theta | k, s (Eq. sam_th): the Gaussian random walk in log space of the
  other samplers, target p(theta) prod_i Poisson(k^i | Omega_theta T^i)
  p(s^i | k^i, theta), with the same prior Normal(1, 1e5) on every log-rate.

Every state probability p(s^i | k^i, theta) comes from mjp_jump_probs (the
paper's algorithm for J-MJP on the GPU: one sweep to max_i k^i per chain,
reading the iterate at each observation's own k^i).  Marginalising the k^i
gives back the exact posterior of theta, so J-MJP and the marginal samplers
agree in distribution; the paper's point (Sec. 3.2.2) is that J-MJP mixes far
worse.  Chain bookkeeping uses torch tensors on the device; random numbers
come from the caller's torch generator.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import mjp
from .sampler import PRIOR_MU, PRIOR_SIGMA


class JumpPosterior:
    """Observations as individual snapshots (a tallied record of count c is c
    observations, each with its own jump count)."""

    def __init__(self, model: int, T, recs, dims, x0=(0, 0), opts=None, n_par: int = 4):
        import torch
        self.torch = torch
        self.model = model
        self.n_par = n_par
        recs = np.asarray(recs, np.int64).reshape(-1, 4)
        single = np.repeat(recs, recs[:, 3], axis=0)
        single[:, 3] = 1
        self.recs = single.astype(np.int32)
        self.I = len(single)
        self.T = np.asarray(T, np.float64)
        self.obs = mjp.make_obs(self.T, self.recs, x0)
        self.T_obs = torch.as_tensor(self.T[single[:, 0]], dtype=torch.float64, device="cuda")
        self.dims = tuple(int(d) for d in dims)
        self.opts = opts or mjp.mjp_opts_default()
        self.n_calls = 0
        self._dims_cache = {}

    def _dims(self, C):
        t = self._dims_cache.get(C)
        if t is None:
            t = self.torch.tensor([list(self.dims)] * C, dtype=self.torch.int32, device="cuda")
            self._dims_cache[C] = t
        return t

    def logphi(self, psi, k):
        """(log p(s^i | k^i, theta) [C, I], Omega_theta [C])."""
        torch = self.torch
        C = psi.shape[0]
        th = torch.zeros((C, 6 if self.model == mjp.MJP_MODEL_AUTOREG else 4), dtype=torch.float64, device="cuda")
        th[:, :self.n_par] = torch.exp(psi)
        out = torch.empty((C, self.I), dtype=torch.float64, device="cuda")
        om = torch.empty(C, dtype=torch.float64, device="cuda")
        mjp.mjp_jump_probs(self.model, th, self._dims(C), self.obs, k.contiguous(), out, om, self.opts)
        self.n_calls += 1
        return out, om

    def log_k_prior(self, k, omega):
        """log Poisson(k^i | Omega_theta T^i) [C, I]."""
        torch = self.torch
        W = omega[:, None] * self.T_obs[None, :]
        kf = k.to(torch.float64)
        return torch.where(W > 0, kf * torch.log(W.clamp_min(1e-300)) - W - torch.lgamma(kf + 1.0),
                           torch.where(kf == 0, torch.zeros_like(kf), torch.full_like(kf, -float("inf"))))

    def logprior(self, psi):
        return (-0.5 * ((psi - PRIOR_MU) / PRIOR_SIGMA) ** 2).sum(dim=1)

    def log_target(self, psi, k, logphi, omega):
        """log p(theta) + sum_i [log p(k^i | theta) + log p(s^i | k^i, theta)]."""
        return self.logprior(psi) + (self.log_k_prior(k, omega) + logphi).sum(dim=1)


@dataclass
class JumpStats:
    steps: int = 0
    theta_accepted: int = 0
    k_accept_rate: float = 0.0
    jump_prob_calls: int = 0
    seconds: float = 0.0


def k_sweep(post: JumpPosterior, psi, k, logphi, omega, gen):
    """One update of every k^i (Eq. sam_k with the SI's Poisson proposal)."""
    torch = post.torch
    rate = (omega[:, None] * post.T_obs[None, :]).expand(k.shape[0], post.I).contiguous()
    kp = torch.poisson(rate, generator=gen).to(torch.int32)
    lp, _ = post.logphi(psi, kp)
    u = torch.rand(k.shape, dtype=torch.float64, device="cuda", generator=gen)
    acc = torch.log(u) < (lp - logphi)
    return torch.where(acc, kp, k), torch.where(acc, lp, logphi), acc


def run_jmjp(post: JumpPosterior, psi0, Z, steps: int, gen, k_burn: int = 20):
    """Gibbs over (psi, k); returns (psi samples [steps, C, d] on the host,
    stats).  The jump counts start from their prior at psi0 and get k_burn
    sweeps at fixed psi0 first."""
    torch = post.torch
    psi = psi0.clone()
    C, d = psi.shape
    Lc = torch.linalg.cholesky(torch.as_tensor(Z, dtype=torch.float64, device="cuda"))
    n0 = post.n_calls
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, omega = post.logphi(psi, torch.zeros((C, post.I), dtype=torch.int32, device="cuda"))
    k = torch.poisson((omega[:, None] * post.T_obs[None, :]).expand(C, post.I).contiguous(),
                      generator=gen).to(torch.int32)
    logphi, omega = post.logphi(psi, k)
    for _ in range(k_burn):
        k, logphi, _ = k_sweep(post, psi, k, logphi, omega, gen)
    lt = post.log_target(psi, k, logphi, omega)
    out = torch.empty((steps, C, d), dtype=torch.float64, device="cuda")
    acc_theta = 0
    acc_k = 0.0
    for h in range(steps):
        k, logphi, ak = k_sweep(post, psi, k, logphi, omega, gen)
        acc_k += float(ak.to(torch.float64).mean().item())
        prop = psi + torch.randn((C, d), dtype=torch.float64, device="cuda", generator=gen) @ Lc.T
        lpp, omp = post.logphi(prop, k)
        ltp = post.log_target(prop, k, lpp, omp)
        u = torch.rand(C, dtype=torch.float64, device="cuda", generator=gen)
        acc = torch.log(u) < (ltp - lt)
        psi = torch.where(acc[:, None], prop, psi)
        logphi = torch.where(acc[:, None], lpp, logphi)
        omega = torch.where(acc, omp, omega)
        lt = torch.where(acc, ltp, lt)
        out[h] = psi
        acc_theta += int(acc.sum().item())
    torch.cuda.synchronize()
    st = JumpStats(steps=steps, theta_accepted=acc_theta, k_accept_rate=acc_k / max(steps, 1),
                   jump_prob_calls=post.n_calls - n0, seconds=time.perf_counter() - t0)
    return out.cpu().numpy(), st


def run_jmjp_device(post: JumpPosterior, psi0, Z, steps: int, seed: int, k_burn: int = 20):
    """run_jmjp with every step on the device (mjp_jmjp_*: Philox draws, the
    jump-count proposals and their prior, the theta step); returns (psi
    samples [steps, C, d] on the host, stats)."""
    import torch
    C, d = psi0.shape
    cfg = mjp.mjp_sampler_cfg_default(model=post.model, dims=post.dims, chains=C, seed=int(seed),
                                      prior_mu=PRIOR_MU, prior_sigma=PRIOR_SIGMA)
    h = mjp.mjp_jmjp_create(cfg, post.obs, post.opts)
    try:
        mjp.mjp_jmjp_set_proposal(h, np.linalg.cholesky(np.asarray(Z, np.float64)))
        psi0 = torch.as_tensor(psi0, dtype=torch.float64, device="cuda").contiguous()
        out = torch.empty((steps, C, d), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mjp.mjp_jmjp_init(h, psi0, k_burn)
        mjp.mjp_jmjp_run(h, steps, out)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        ctr = mjp.mjp_jmjp_counters(h)
    finally:
        mjp.mjp_jmjp_destroy(h)
    st = JumpStats(steps=steps, theta_accepted=int(ctr[1]), k_accept_rate=float(ctr[2]) / max(float(ctr[3]), 1.0),
                   jump_prob_calls=2 * steps + 3 + k_burn, seconds=sec)
    return out.cpu().numpy(), st
