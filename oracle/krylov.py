"""FP64 CPU oracle of the Krylov-subspace propagator (Method #5 of Pessoa,
Schweiger, Presse, arXiv 2312.05647, Sec. 2.2.5, Algorithm ArnoldiKrylov and
Eq. Krylov_expansion): TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

What is computed, in the paper's order and notation:

* one step over [t, t + dt] starts from q_1 = rho(t) / ||rho(t)||_2 and builds
  q_2 .. q_kappa by Arnoldi with modified Gram-Schmidt: q_i = q_{i-1} A, then
  for j < i  h_{j,i-1} = <q_j, q_i>, q_i -= h_{j,i-1} q_j; h_{i,i-1} = ||q_i||,
  q_i /= h_{i,i-1}.  That is kappa - 1 products with A, and H is kappa x kappa
  with its last column zero (the algorithm never forms q_kappa A);
* rho(t + dt) = ||rho(t)||_2 * sum_i [exp(H dt)]_{i,1} q_i  (first column of
  the small exponential, mapped back through the basis);
* dt = dt_factor * kappa / max_n |a_nn|, with dt_factor = 2 the paper's
  choice; the last step before each requested time is shortened so the
  propagation lands on it.

Readings where the paper is silent (stated again in the design notes):

* breakdown: if h_{i,i-1} <= 1e-12 ||q_{i-1} A||_2 the subspace is (to
  rounding) invariant; the basis stops at i - 1 vectors and the remaining
  rows and columns of H are zero, which leaves exp(H dt) e_1 on the
  invariant subspace unchanged;
* several output times: one propagation through the sorted times.

Library primitives used as single steps: ``scipy.sparse`` products with A^T
(rho is a row vector, rho A = (A^T rho^T)^T) and ``scipy.linalg.expm`` for
the kappa x kappa exponential (Pade 13 with scaling and squaring).

Parity status: pinned by tests/test_oracle_krylov.py (invariant-subspace
cases against scipy.linalg.expm, a two-state closed form, Arnoldi relations,
mass conservation, convergence to the exact R-MJP oracle as dt shrinks).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sl
import scipy.sparse as sp

BREAKDOWN_REL = 1e-12


def _transpose(A):
    """A^T as a scipy CSR matrix from the oracle's CSR (row = from-state)."""
    M = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    return M.T.tocsr()


def max_exit_rate(A) -> float:
    """m_theta = max_n |a_nn| (Eq. A_def: the diagonal holds minus the exit rate)."""
    d = np.zeros(A.n)
    for r in range(A.n):
        for e in range(A.row_ptr[r], A.row_ptr[r + 1]):
            if A.col[e] == r:
                d[r] += A.val[e]
    return float(np.abs(d).max()) if A.n else 0.0


def arnoldi(At, rho, kappa: int):
    """Algorithm ArnoldiKrylov: returns (beta, Q [m x N], H [kappa x kappa], m)
    where m <= kappa is the basis size actually built (m < kappa after a
    breakdown); rows of Q are the basis vectors q_1 .. q_m."""
    beta = float(np.linalg.norm(rho))
    N = rho.size
    Q = np.zeros((kappa, N))
    H = np.zeros((kappa, kappa))
    if beta == 0.0:
        return beta, Q[:0], H, 0
    Q[0] = rho / beta
    m = kappa
    for i in range(1, kappa):
        w = At @ Q[i - 1]
        wnorm = float(np.linalg.norm(w))
        for j in range(i):
            H[j, i - 1] = float(Q[j] @ w)
            w = w - H[j, i - 1] * Q[j]
        h = float(np.linalg.norm(w))
        if h <= BREAKDOWN_REL * wnorm or h == 0.0:
            m = i
            break
        H[i, i - 1] = h
        Q[i] = w / h
    return beta, Q[:m], H, m


def krylov_step(At, rho, dt: float, kappa: int):
    """One step of Eq. Krylov_expansion."""
    beta, Q, H, m = arnoldi(At, rho, kappa)
    if m == 0:
        return np.zeros_like(rho)
    E = sl.expm(H[:m, :m] * dt)
    return beta * (E[:, 0] @ Q)


def krylov_expv(A, rho0, times, kappa: int = 20, dt_factor: float = 2.0):
    """rho0 exp(A t) for each t in `times` (any order); returns
    (out [len(times) x N], info) with info = {m_theta, dt, steps}."""
    times = np.asarray(times, np.float64)
    At = _transpose(A)
    mth = max_exit_rate(A)
    rho = np.asarray(rho0, np.float64).copy()
    out = np.zeros((len(times), rho.size))
    if mth == 0.0:
        out[:] = rho
        return out, {"m_theta": 0.0, "dt": math.inf, "steps": 0}
    dt = dt_factor * kappa / mth
    tau, steps = 0.0, 0
    for idx in np.argsort(times, kind="stable"):
        t = float(times[idx])
        while t - tau > 0.0:
            h = min(dt, t - tau)
            rho = krylov_step(At, rho, h, kappa)
            tau = t if h == t - tau else tau + h
            steps += 1
        out[idx] = rho
    return out, {"m_theta": mth, "dt": dt, "steps": steps}
