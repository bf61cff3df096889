"""FP64 CPU oracle of the jump-based method J-MJP (Method #2 of Pessoa,
Schweiger, Presse, arXiv 2312.05647, Sec. 2.2.2, Algorithm "State
probabilities for J-MJP", Eq. sample_J-MJP; the jump-count proposal of the
SI): TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

J-MJP keeps, for every observation i (one system observed in state s^i at
time T^i), the number k^i of virtual jumps of the uniformised chain up to
T^i as a latent variable.  Given k^i the state probability is a plain power
of B = I + A/Omega (Omega = 1.1 max|a_nn|, Eq. B_def):

    p(s^i | k^i, theta) = (rho(0) B^{k^i})_{s^i},

and k^i has the prior p(k^i | theta) = Poisson(k^i | Omega_theta T^i)
(Eq. ME_uniform).  The Gibbs sampler alternates k | s, theta and
theta | k, s (Eqs. sam_k, sam_th).

* ``state_probs`` -- the algorithm: one sweep of rho <- rho B up to
  max_i k^i, reading rho at s^i when the sweep reaches k^i.  s^i may be a
  group of state indices (a hidden gene state, summed as in Sec. 3.1.2).
* ``log_prior_k`` -- log Poisson(k | Omega T).
* ``k_conditional`` -- p(k | s, theta), normalised over k = 0..kmax.
* ``log_joint`` -- log p(k | theta) + log p(s | k, theta), the theta-dependent
  part of the target of Eq. sam_th besides the prior.

The jump product is ``oracle.jump`` (the same FP64 step as Algorithm 2).

Parity status: pinned by tests/test_oracle_jmjp.py (the Poisson mixture of
the state probabilities over k equals scipy's matrix exponential; a pure
birth chain's jump-count probabilities are binomial; k = 0 returns rho(0);
mass; hidden-state groups).
"""
from __future__ import annotations

import math

import numpy as np

from . import CSR, jump


def omega(A: CSR, omega_factor: float = 1.1) -> float:
    """Omega_theta = omega_factor * max_n |a_nn| (Eq. B_def)."""
    m = 0.0
    for r in range(A.n):
        for e in range(A.row_ptr[r], A.row_ptr[r + 1]):
            if A.col[e] == r:
                m = max(m, abs(float(A.val[e])))
    return omega_factor * m


def state_probs(A: CSR, rho0, groups, ks, omega_factor: float = 1.1) -> np.ndarray:
    """phi[i] = sum_{s in groups[i]} (rho(0) B^{ks[i]})_s."""
    ks = np.asarray(ks, dtype=np.int64)
    phi = np.zeros(len(ks))
    if len(ks) == 0:
        return phi
    rho = np.asarray(rho0, dtype=np.float64).copy()
    kmax = int(ks.max())
    pending = {}
    for i, k in enumerate(ks):
        pending.setdefault(int(k), []).append(i)
    k = 0
    while k <= kmax:
        for i in pending.get(k, []):
            phi[i] = float(np.sum(rho[np.asarray(groups[i], dtype=np.int64)]))
        k += 1
        if k <= kmax:
            rho = jump(A, rho, omega_factor)
    return phi


def log_prior_k(k, omega_theta: float, T: float) -> float:
    """log Poisson(k | Omega_theta T)."""
    W = omega_theta * T
    if W == 0.0:
        return 0.0 if k == 0 else -math.inf
    return k * math.log(W) - W - math.lgamma(k + 1.0)


def k_conditional(A: CSR, rho0, group, T: float, kmax: int, omega_factor: float = 1.1) -> np.ndarray:
    """p(k | s, theta) for k = 0..kmax (Eq. sam_k), normalised on that range."""
    om = omega(A, omega_factor)
    phi = state_probs(A, rho0, [group] * (kmax + 1), np.arange(kmax + 1), omega_factor)
    lp = np.array([log_prior_k(k, om, T) for k in range(kmax + 1)])
    w = np.exp(lp - lp.max()) * phi
    return w / w.sum()


def log_joint(A: CSR, rho0, groups, ks, T_obs, omega_factor: float = 1.1) -> float:
    """sum_i [log Poisson(k^i | Omega T^i) + log p(s^i | k^i, theta)]."""
    om = omega(A, omega_factor)
    phi = state_probs(A, rho0, groups, ks, omega_factor)
    if np.any(phi <= 0.0):
        return -math.inf
    return float(sum(log_prior_k(int(k), om, float(t)) for k, t in zip(ks, T_obs)) + np.log(phi).sum())
