"""FP64 CPU oracle of the fourth-order Runge-Kutta propagator (Method #4 of
Pessoa, Schweiger, Presse, arXiv 2312.05647, Sec. 2.2.4, Eqs. RKstep and
RKintermediate): TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

The method integrates d rho / dt = rho A(t) with the classical RK4 step

    d1 = dt rho(t) A(t)
    d2 = dt (rho(t) + d1/2) A(t + dt/2)
    d3 = dt (rho(t) + d2/2) A(t + dt/2)
    d4 = dt (rho(t) + d3) A(t + dt)
    rho(t + dt) = rho(t) + (d1 + 2 d2 + 2 d3 + d4) / 6,

which allows rates that change in time (the paper's reason to keep it).
Time dependence is written as A(t) = sum_c g_c(t) A_c: each channel A_c is a
generator (non-negative off-diagonal rates, rows summing to 0) and g_c(t) >= 0
is piecewise linear through given knots (constant outside them), so A(t) is a
generator at every t.

Readings where the paper is silent (stated again in the design notes):
* step: dt = dt_factor / m with m = max over t of max_n |a_nn(t)| (the paper's
  stability condition dt <= 1/max|a_nn| is dt_factor = 1); m is attained at a
  knot, because max_n |a_nn(t)| is convex in the g_c and the g_c are linear
  between knots;
* the last step before each requested time is shortened to land on it.

Library primitive used as a step: ``scipy.sparse`` products with A_c^T.

Parity status: pinned by tests/test_oracle_rk4.py (one step equals the
fourth-order Taylor polynomial of exp(A dt) for constant A; fourth-order
convergence to the exact R-MJP oracle; immigration-death with a time-varying
birth rate against its Poisson closed form; a two-state chain with
time-scaled rates against its closed form; mass conservation).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class Schedule:
    """Piecewise-linear g(t) through knots (t_k, v_k), constant outside."""

    def __init__(self, t_knots=(0.0,), values=(1.0,)):
        self.t = np.asarray(t_knots, np.float64)
        self.v = np.asarray(values, np.float64)

    def __call__(self, t: float) -> float:
        return float(np.interp(t, self.t, self.v))


def _transpose(A):
    return sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n)).T.tocsr()


def _diag(A):
    d = np.zeros(A.n)
    for r in range(A.n):
        for e in range(A.row_ptr[r], A.row_ptr[r + 1]):
            if A.col[e] == r:
                d[r] += A.val[e]
    return d


def max_exit_rate(channels, schedules) -> float:
    """max over the knots of max_n |sum_c g_c(t) a^c_nn|."""
    diags = [np.abs(_diag(A)) for A in channels]
    knots = np.unique(np.concatenate([s.t for s in schedules]))
    return max(float(np.max(sum(s(t) * d for s, d in zip(schedules, diags)))) for t in knots)


def rk4_expv(channels, schedules, rho0, times, dt_factor: float = 1.0):
    """rho0 propagated to each t in `times` (any order); returns
    (out [len(times) x N], info) with info = {m, dt, steps}."""
    Ats = [_transpose(A) for A in channels]
    m = max_exit_rate(channels, schedules)
    rho = np.asarray(rho0, np.float64).copy()
    times = np.asarray(times, np.float64)
    out = np.zeros((len(times), rho.size))
    if m == 0.0:
        out[:] = rho
        return out, {"m": 0.0, "dt": np.inf, "steps": 0}
    dt = dt_factor / m

    def prod(x, t):  # x A(t)
        return sum(s(t) * (At @ x) for s, At in zip(schedules, Ats))

    tau, steps = 0.0, 0
    for idx in np.argsort(times, kind="stable"):
        t_end = float(times[idx])
        while t_end - tau > 0.0:
            h = min(dt, t_end - tau)
            d1 = h * prod(rho, tau)
            d2 = h * prod(rho + d1 / 2, tau + h / 2)
            d3 = h * prod(rho + d2 / 2, tau + h / 2)
            d4 = h * prod(rho + d3, tau + h)
            rho = rho + (d1 + 2 * d2 + 2 * d3 + d4) / 6
            tau = t_end if h == t_end - tau else tau + h
            steps += 1
        out[idx] = rho
    return out, {"m": m, "dt": dt, "steps": steps}
