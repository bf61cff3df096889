"""Posterior samplers over log-rates psi = log(theta), batched over chains.

* Metropolis-Hastings with a Gaussian random walk in log space and the prior
  Normal(mu = 1, sigma = 1e5) on every log-rate (SI: sampling scheme and
  prior); every proposal is scored by the exact log-likelihood (mjp_loglik,
  the R-MJP expansion on the GPU).
* Delayed acceptance (Christen and Fox, J. Comput. Graph. Stat. 14(4), 2005):
  a cheap screen (the MLP surrogate) accepts or rejects first; only the
  proposals it accepts are scored exactly, and a second test with the ratio
  of exact to screened posterior ratios keeps the exact posterior invariant.
* Proposal covariance by the SI's adaptive scheme
  Z = (2.38 / eta)^2 (cov + eps I), pooled over chains, then frozen so both
  samplers share it.

The random numbers (proposal normals, acceptance uniforms) are drawn by the
caller's torch generator and passed through, so a run is reproducible and two
samplers fed the same draws can be compared path by path.  Chain
bookkeeping (proposals, acceptance, compaction) uses torch tensors on the
device; every likelihood and surrogate evaluation runs in libmjp's kernels.
"""
from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import mjp

PRIOR_MU = 1.0
PRIOR_SIGMA = 1e5


class Posterior:
    """log p(psi | data) up to a constant for a built-in model on a fixed grid."""

    def __init__(self, model: int, T, recs, dims, x0=(0, 0), opts=None, n_par: int = 4):
        import torch
        self.torch = torch
        self.model = model
        self.n_par = n_par
        self.obs = mjp.make_obs(np.asarray(T, np.float64), np.asarray(recs, np.int32).reshape(-1, 4), x0)
        self.dims = tuple(int(d) for d in dims)
        self.opts = opts or mjp.mjp_opts_default()
        self.n_exact = 0
        self._dims_cache = {}

    def _dims(self, B):
        t = self._dims_cache.get(B)
        if t is None:
            t = self.torch.tensor([list(self.dims)] * B, dtype=self.torch.int32, device="cuda")
            self._dims_cache[B] = t
        return t

    def loglik(self, psi):
        torch = self.torch
        B = psi.shape[0]
        out = torch.empty(B, dtype=torch.float64, device="cuda")
        if B == 0:
            return out
        th = torch.zeros((B, 4), dtype=torch.float64, device="cuda")
        th[:, :self.n_par] = torch.exp(psi)
        mjp.mjp_loglik(self.model, th, self._dims(B), self.obs, out, self.opts)
        self.n_exact += B
        return out

    def logprior(self, psi):
        return (-0.5 * ((psi - PRIOR_MU) / PRIOR_SIGMA) ** 2).sum(dim=1)

    def logpost(self, psi):
        return self.loglik(psi) + self.logprior(psi)


class SurrogateScreen:
    """Standardised MLP surrogate of the log-likelihood: the screen of the
    delayed-acceptance sampler (log-prior added exactly)."""

    def __init__(self, handle, psi_mean, psi_std, ll_mean, ll_std):
        import torch
        self.torch = torch
        self.h = handle
        self.psi_mean = torch.as_tensor(psi_mean, dtype=torch.float64, device="cuda")
        self.psi_std = torch.as_tensor(psi_std, dtype=torch.float64, device="cuda")
        self.ll_mean, self.ll_std = float(ll_mean), float(ll_std)
        self.n_eval = 0

    def __call__(self, psi):
        torch = self.torch
        x = ((psi - self.psi_mean) / self.psi_std).float().contiguous()
        y = torch.empty(psi.shape[0], dtype=torch.float32, device="cuda")
        mjp.mjp_surrogate_infer(self.h, x, y)
        self.n_eval += psi.shape[0]
        ll = y.double() * self.ll_std + self.ll_mean
        return ll + (-0.5 * ((psi - PRIOR_MU) / PRIOR_SIGMA) ** 2).sum(dim=1)


def train_surrogate(psi, ll, width=256, depth=3, epochs=60, batch=1024, lr=2e-3, seed=0):
    """Fit the MLP to (psi, exact log-likelihood) pairs; returns the screen
    and the per-epoch training losses (standardised units)."""
    import torch
    psi = torch.as_tensor(psi, dtype=torch.float64, device="cuda")
    ll = torch.as_tensor(ll, dtype=torch.float64, device="cuda")
    m, s = psi.mean(0), psi.std(0)
    lm, ls = ll.mean().item(), ll.std().item()
    x = ((psi - m) / s).float().contiguous()
    y = ((ll - lm) / ls).float().contiguous()
    h = mjp.mjp_surrogate_create(psi.shape[1], width, depth, seed=seed)
    cfg = mjp.mjp_train_cfg_default(epochs=epochs, batch=batch, lr=lr, seed=seed)
    t0 = time.perf_counter()
    losses = mjp.mjp_surrogate_train(h, x, y, cfg)
    torch.cuda.synchronize()
    return SurrogateScreen(h, m, s, lm, ls), losses, time.perf_counter() - t0


@dataclass
class ChainStats:
    steps: int = 0
    accepted: int = 0
    stage1_accepted: int = 0
    exact_evals: int = 0
    screen_evals: int = 0
    seconds: float = 0.0
    extra: dict = field(default_factory=dict)


def _draws(gen, steps, C, d):
    import torch
    z = torch.randn((steps, C, d), dtype=torch.float64, device="cuda", generator=gen)
    u = torch.rand((steps, C, 2), dtype=torch.float64, device="cuda", generator=gen)
    return z, u


def run_mh(post: Posterior, psi0, Z, steps: int, gen, draws=None, progress=None):
    """Plain Metropolis-Hastings; returns (samples [steps, C, d] on the host, stats).
    progress, if given, is called with the step number after every 10th step."""
    import torch
    psi = psi0.clone()
    C, d = psi.shape
    Lc = torch.linalg.cholesky(torch.as_tensor(Z, dtype=torch.float64, device="cuda"))
    z, u = draws if draws is not None else _draws(gen, steps, C, d)
    n0 = post.n_exact
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lp = post.logpost(psi)
    out = torch.empty((steps, C, d), dtype=torch.float64, device="cuda")
    acc_total = 0
    for h in range(steps):
        prop = psi + z[h] @ Lc.T
        lpp = post.logpost(prop)
        acc = torch.log(u[h, :, 0]) < (lpp - lp)
        psi = torch.where(acc[:, None], prop, psi)
        lp = torch.where(acc, lpp, lp)
        out[h] = psi
        acc_total += int(acc.sum().item())
        if progress is not None and (h + 1) % 10 == 0:
            progress(h + 1)
    torch.cuda.synchronize()
    st = ChainStats(steps=steps, accepted=acc_total, exact_evals=post.n_exact - n0,
                    seconds=time.perf_counter() - t0)
    return out.cpu().numpy(), st


def run_da(post: Posterior, screen, psi0, Z, steps: int, gen, draws=None, progress=None):
    """Delayed-acceptance Metropolis-Hastings with `screen` (a callable
    returning a screened log-posterior) as the first stage.  progress as in
    run_mh."""
    import torch
    psi = psi0.clone()
    C, d = psi.shape
    Lc = torch.linalg.cholesky(torch.as_tensor(Z, dtype=torch.float64, device="cuda"))
    z, u = draws if draws is not None else _draws(gen, steps, C, d)
    n0 = post.n_exact
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lp = post.logpost(psi)
    sc = screen(psi)
    out = torch.empty((steps, C, d), dtype=torch.float64, device="cuda")
    acc_total = s1_total = scr = 0
    for h in range(steps):
        prop = psi + z[h] @ Lc.T
        scp = screen(prop)
        scr += C
        a1 = torch.log(u[h, :, 0]) < (scp - sc)
        idx = torch.nonzero(a1).flatten()
        s1_total += int(idx.numel())
        if idx.numel():
            lpp = post.logpost(prop[idx])
            a2 = torch.log(u[h, idx, 1]) < (lpp - lp[idx]) - (scp[idx] - sc[idx])
            take = idx[a2]
            psi[take] = prop[take]
            lp[take] = lpp[a2]
            sc[take] = scp[take]
            acc_total += int(take.numel())
        out[h] = psi
        if progress is not None and (h + 1) % 10 == 0:
            progress(h + 1)
    torch.cuda.synchronize()
    st = ChainStats(steps=steps, accepted=acc_total, stage1_accepted=s1_total,
                    exact_evals=post.n_exact - n0, screen_evals=scr, seconds=time.perf_counter() - t0)
    return out.cpu().numpy(), st


class DeviceChains:
    """Chains whose every step runs on the device (mjp_sampler_*): Philox
    draws keyed by `seed`, stage 1, the masked exact likelihood and the
    accept step as one fixed sequence of launches with no host read.  With a
    screen the chains use delayed acceptance, else plain MH; the same seed,
    start and covariance give the same chains, and plain MH equals delayed
    acceptance under a constant screen."""

    def __init__(self, post: Posterior, chains: int, seed: int, Z, screen: SurrogateScreen | None = None):
        import torch
        self.torch = torch
        npar = 2 if post.model == mjp.MJP_MODEL_BD else (6 if post.model == mjp.MJP_MODEL_AUTOREG else 4)
        assert post.n_par == npar, "the device sampler samples all of the model's log-rates"
        self.C, self.d = int(chains), npar
        cfg = mjp.mjp_sampler_cfg_default(model=post.model, dims=post.dims, chains=self.C, seed=int(seed),
                                          prior_mu=PRIOR_MU, prior_sigma=PRIOR_SIGMA)
        self.h = mjp.mjp_sampler_create(cfg, post.obs, post.opts)
        mjp.mjp_sampler_set_proposal(self.h, np.linalg.cholesky(np.asarray(Z, np.float64)))
        if screen is not None:
            mjp.mjp_sampler_set_screen(self.h, screen.h, screen.psi_mean.cpu().numpy(), screen.psi_std.cpu().numpy(),
                                       screen.ll_mean, screen.ll_std)

    def init(self, psi0, stream=None):
        psi0 = self.torch.as_tensor(psi0, dtype=self.torch.float64, device="cuda").contiguous()
        mjp.mjp_sampler_init(self.h, psi0, stream=stream)

    def run(self, steps: int, samples=None, stream=None):
        mjp.mjp_sampler_run(self.h, steps, samples, stream=stream)

    def state(self):
        return mjp.mjp_sampler_get_state(self.h, self.C, self.d)

    def set_state(self, st):
        mjp.mjp_sampler_set_state(self.h, st)

    def close(self):
        if self.h:
            mjp.mjp_sampler_destroy(self.h)
            self.h = None


def run_device(post: Posterior, psi0, Z, steps: int, seed: int, screen: SurrogateScreen | None = None,
               progress=None):
    """run_mh (screen None) or run_da on the device; returns (samples
    [steps, C, d] on the host, stats).  progress as in run_mh."""
    import torch
    ch = DeviceChains(post, psi0.shape[0], seed, Z, screen)
    try:
        samples = torch.empty((steps, ch.C, ch.d), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.init(psi0)
        done = 0
        while done < steps:
            n = min(10, steps - done)
            ch.run(n, samples)  # the ring is the whole array: row h after step h
            done += n
            if progress is not None and done % 10 == 0:
                torch.cuda.synchronize()
                progress(done)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        ctr = ch.state()["counters"]
    finally:
        ch.close()
    st = ChainStats(steps=steps, accepted=int(ctr[1]), stage1_accepted=int(ctr[2]),
                    exact_evals=int(ctr[3]) + psi0.shape[0], screen_evals=(steps + 1) * psi0.shape[0] if screen else 0,
                    seconds=sec)
    return samples.cpu().numpy(), st


def adapt_covariance(post: Posterior, psi0, gen, rounds: int = 6, steps: int = 40, z0: float = 1e-4,
                     eps: float = 1e-12, final_scale: str = "si"):
    """SI adaptive scheme: Z = (2.38 / eta)^2 [cov(recent samples) + eps I],
    the covariance pooled over all chains' last `steps` samples, `rounds`
    times.  final_scale "si" returns that Z; "optimal" returns the same
    pooled covariance scaled by 2.38^2 / eta (the random-walk scaling of
    Gelman, Roberts and Gilks), which the SI's constant is 1/eta of.
    Returns (Z, last states)."""
    import torch
    C, d = psi0.shape
    Z = z0 * np.eye(d)
    psi = psi0
    cov = None
    for _ in range(rounds):
        s, st = run_mh(post, psi, Z, steps, gen)
        flat = s.reshape(-1, d)
        cov = np.cov(flat.T) + eps * np.eye(d)
        Z = (2.38 / d) ** 2 * cov
        psi = torch.as_tensor(s[-1], device="cuda")
    if final_scale == "optimal":
        Z = 2.38 ** 2 / d * cov
    return Z, psi


def autocorrelation(x):
    """ACF of a 1-D chain (the paper's Eq. autocorr with the mean taken as
    (1/H) sum; lag-tau products averaged over H - tau terms)."""
    x = np.asarray(x, np.float64)
    H = len(x)
    xc = x - x.mean()
    f = np.fft.rfft(xc, n=2 * H)
    acov = np.fft.irfft(f * np.conj(f))[:H] / (H - np.arange(H))
    return acov / acov[0] if acov[0] > 0 else np.zeros(H)


def ess(samples):
    """Effective sample size per parameter, summed over chains: each chain's
    integrated autocorrelation time from Geyer's initial positive sequence
    of paired ACF sums.  samples: [steps, chains, d]."""
    S, C, d = samples.shape
    out = np.zeros(d)
    for j in range(d):
        tot = 0.0
        for c in range(C):
            rho = autocorrelation(samples[:, c, j])
            tau = -1.0
            for m in range(S // 2):
                g = rho[2 * m] + rho[2 * m + 1] if 2 * m + 1 < S else rho[2 * m]
                if not g > 0:
                    break
                tau += 2 * g
            tot += S / max(tau, 1.0)
        out[j] = tot
    return out
