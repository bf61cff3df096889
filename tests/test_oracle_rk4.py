"""Pins for the FP64 RK4 oracle (Method #4, Eqs. RKstep / RKintermediate)
against facts independent of its code:

* for constant A one RK4 step is the fourth-order Taylor polynomial of
  exp(A dt): rho (I + hA + (hA)^2/2 + (hA)^3/6 + (hA)^4/24);
* the global error falls ~16x when dt halves (fourth order), towards the
  exact R-MJP oracle;
* immigration-death with a piecewise-linear birth rate beta g(t) stays
  Poisson with mean m(t), dm/dt = beta g(t) - gamma m, solved exactly per
  linear segment;
* a two-state chain whose switching rates are scaled by g(t) has the active
  probability a + (p0 - a) exp(-(l_act + l_ina) G(t)), G = int_0^t g;
* mass is conserved.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl
from scipy.stats import poisson

import oracle
from oracle import rk4
from paper_2312_05647_amd import synth


def test_one_step_is_fourth_order_taylor():
    rp, ci, va = synth.with_generator_diagonal(*synth.random_rate_graph(12, 4, dense=True, scale=2.0))
    A = oracle.CSR.from_arrays(rp, ci, va)
    rho0 = synth.random_prob(12, 3)
    h = 0.9 / rk4.max_exit_rate([A], [rk4.Schedule()])
    got, info = rk4.rk4_expv([A], [rk4.Schedule()], rho0, [h], dt_factor=0.9)
    assert info["steps"] == 1
    M = A.dense() * h
    T = np.eye(12) + M + M @ M / 2 + M @ M @ M / 6 + M @ M @ M @ M / 24
    assert np.abs(got[0] - rho0 @ T).max() < 1e-15


def test_fourth_order_convergence():
    A = oracle.model_generator(oracle.MODEL_BD, [80.0, 1.0], [300])
    rho0 = synth.delta(300)
    exact, _ = oracle.expv(A, rho0, 1.0, eps_right=1e-15)
    err = []
    for f in (1.0, 0.5, 0.25):
        got, _ = rk4.rk4_expv([A], [rk4.Schedule()], rho0, [1.0], dt_factor=f)
        err.append(np.abs(got[0] - exact).sum())
        assert abs(got[0].sum() - 1.0) < 1e-12
    assert 10.0 < err[0] / err[1] < 22.0 and 10.0 < err[1] / err[2] < 22.0, err


def poisson_mean_piecewise(beta, gamma, knots_t, knots_g, t):
    """Exact m(t) for dm/dt = beta g(t) - gamma m, m(0) = 0, g piecewise
    linear through the knots (constant outside)."""
    pts = sorted(set([0.0, t] + [k for k in knots_t if 0.0 < k < t]))
    m = 0.0
    for t0, t1 in zip(pts[:-1], pts[1:]):
        g0, g1 = np.interp(t0, knots_t, knots_g), np.interp(t1, knots_t, knots_g)
        b = beta * (g1 - g0) / (t1 - t0)          # forcing a + b (s - t0)
        a = beta * g0
        mp0 = a / gamma - b / gamma ** 2           # particular solution at t0
        mp1 = mp0 + (b / gamma) * (t1 - t0)
        m = mp1 + (m - mp0) * math.exp(-gamma * (t1 - t0))
    return m


def test_time_varying_birth_rate_is_poisson():
    beta, gamma, N = 120.0, 1.0, 600
    birth = oracle.model_generator(oracle.MODEL_BD, [beta, 0.0], [N])
    death = oracle.model_generator(oracle.MODEL_BD, [0.0, gamma], [N])
    kt, kg = [0.0, 0.5, 1.5, 2.0], [0.2, 1.0, 3.0, 0.5]
    sched = [rk4.Schedule(kt, kg), rk4.Schedule()]
    times = [0.25, 1.0, 2.5]
    got, info = rk4.rk4_expv([birth, death], sched, synth.delta(N), times, dt_factor=0.25)
    for j, t in enumerate(times):
        mean = poisson_mean_piecewise(beta, gamma, kt, kg, t)
        ref = poisson.pmf(np.arange(N), mean)
        assert np.abs(got[j] - ref).sum() < 1e-8, (t, np.abs(got[j] - ref).sum())


def test_time_scaled_switching_closed_form():
    beta, gamma, lact, lina, NR = 40.0, 1.0, 2.0, 1.0, 120
    prod = oracle.model_generator(oracle.MODEL_TWOSTATE, [beta, gamma, 0.0, 0.0], [NR])
    switch = oracle.model_generator(oracle.MODEL_TWOSTATE, [0.0, 0.0, lact, lina], [NR])
    kt, kg = [0.0, 1.0, 2.0], [0.5, 2.0, 1.0]
    sched = [rk4.Schedule(), rk4.Schedule(kt, kg)]
    t = 2.5
    got, _ = rk4.rk4_expv([prod, switch], sched, synth.delta(2 * NR), [t], dt_factor=0.25)
    G = 0.5 * (0.5 + 2.0) * 1.0 + 0.5 * (2.0 + 1.0) * 1.0 + 1.0 * 0.5   # integral of g over [0, 2.5]
    a = lact / (lact + lina)
    p_act = a + (1.0 - a) * math.exp(-(lact + lina) * G)
    assert abs(got[0][:NR].sum() - p_act) < 1e-9
    assert abs(got[0].sum() - 1.0) < 1e-12


def test_trivial_cases():
    A = oracle.model_generator(oracle.MODEL_BD, [5.0, 1.0], [30])
    rho0 = synth.random_prob(30, 1)
    got, info = rk4.rk4_expv([A], [rk4.Schedule()], rho0, [0.0])
    assert np.array_equal(got[0], rho0) and info["steps"] == 0
    got, info = rk4.rk4_expv([A], [rk4.Schedule([0.0], [0.0])], rho0, [2.0])   # g = 0: A(t) = 0
    assert np.array_equal(got[0], rho0)
