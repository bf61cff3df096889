"""Pins for the FP64 Krylov oracle (Method #5, Algorithm ArnoldiKrylov and
Eq. Krylov_expansion) against facts that do not come from the oracle itself:

* when the Krylov subspace is invariant (N < kappa, or a two-state chain)
  the step is exact, so the result equals the dense exponential
  (scipy.linalg.expm) and the two-state closed form;
* the Arnoldi relations: the basis is orthonormal and H holds the projections
  <q_j, q_i A> of the products the algorithm forms;
* rows of A sum to zero, so A 1 = 0 and every step keeps sum(rho);
* as dt shrinks the result converges to the exact R-MJP oracle (1e-12);
* the paper's dt = 2 kappa / m_theta gives a stable but inexact propagator:
  its error at the C1 workload stays within 5e-3 (measured 2.2e-3).
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from oracle import krylov
from paper_2312_05647_amd import synth


def dense_expv(A, rho0, t):
    return np.asarray(rho0, np.float64) @ sl.expm(A.dense() * t)


def test_invariant_subspace_is_exact():
    """N = 8 < kappa: Arnoldi breaks down by N vectors; the step is exact."""
    rp, ci, va = synth.with_generator_diagonal(*synth.random_rate_graph(8, 3, dense=True, scale=2.0))
    A = oracle.CSR.from_arrays(rp, ci, va)
    rho0 = synth.random_prob(8, 5)
    times = [0.0, 0.3, 1.7, 5.0]
    got, info = krylov.krylov_expv(A, rho0, times, kappa=20)
    for j, t in enumerate(times):
        assert np.abs(got[j] - dense_expv(A, rho0, t)).max() < 1e-12


def test_two_state_closed_form():
    """a: 0 -> 1 at rate a, 1 -> 0 at rate b; p0(t) = b/(a+b) + (p0(0) - b/(a+b)) e^{-(a+b) t}."""
    a, b = 3.0, 1.25
    A = oracle.CSR.from_arrays([0, 2, 4], [0, 1, 0, 1], [-a, a, b, -b])
    for t in (0.1, 0.9, 4.0):
        got, _ = krylov.krylov_expv(A, [0.7, 0.3], [t], kappa=20, dt_factor=2.0)
        p0 = b / (a + b) + (0.7 - b / (a + b)) * math.exp(-(a + b) * t)
        assert abs(got[0, 0] - p0) < 1e-14 and abs(got[0, 1] - (1 - p0)) < 1e-14


def test_arnoldi_relations():
    A = oracle.model_generator(oracle.MODEL_CASCADE2, [20.0, 1.0, 0.5, 0.5], [40, 30])
    At = krylov._transpose(A)
    rho = synth.random_prob(1200, 9)
    beta, Q, H, m = krylov.arnoldi(At, rho, 20)
    assert m == 20 and abs(beta - np.linalg.norm(rho)) < 1e-15
    assert np.abs(Q @ Q.T - np.eye(m)).max() < 1e-12
    Ad = A.dense()
    # column i-1 of H holds <q_j, q_{i-1} A> for j <= i; the last column is never formed
    P = (Q @ Ad) @ Q.T  # P[i, j] = <q_j, q_i A>
    for i in range(1, m):
        for j in range(i + 1):
            assert abs(H[j, i - 1] - P[i - 1, j]) < 1e-10 * max(1.0, abs(P[i - 1, j]))
    assert np.all(H[:, m - 1] == 0.0)
    assert np.all(np.tril(H, -2) == 0.0)  # upper Hessenberg


def test_mass_is_kept():
    A = oracle.model_generator(oracle.MODEL_BD, [500.0, 1.0], [1000])
    got, info = krylov.krylov_expv(A, synth.random_prob(1000, 2), [0.2, 1.0], kappa=20)
    assert np.abs(got.sum(axis=1) - 1.0).max() < 1e-12


def test_converges_to_exact_as_dt_shrinks():
    A = oracle.model_generator(oracle.MODEL_BD, [500.0, 1.0], [1000])
    rho0 = synth.delta(1000)
    exact, _ = oracle.expv(A, rho0, 1.0, eps_right=1e-15)
    err = {}
    for f in (2.0, 1.0, 0.5):
        got, info = krylov.krylov_expv(A, rho0, [1.0], kappa=20, dt_factor=f)
        err[f] = np.abs(got[0] - exact).sum()
        assert info["steps"] == math.ceil(1.0 / info["dt"])
    assert err[2.0] < 5e-3          # the paper's step: stable, L1 ~2e-3 here
    assert err[1.0] < err[2.0] * 1e-2
    assert err[0.5] < 1e-9


def test_cascade_against_exact_at_half_step():
    A = oracle.model_generator(oracle.MODEL_CASCADE2, [20.0, 1.0, 0.5, 0.5], [40, 30])
    rho0 = synth.delta(1200)
    times = [0.5, 3.0, 1.0]
    got, _ = krylov.krylov_expv(A, rho0, times, kappa=20, dt_factor=0.5)
    ref = oracle.expv_times(A, rho0, times, eps_right=1e-15)
    assert np.abs(got - ref).sum(axis=1).max() < 1e-11


def test_trivial_cases():
    A = oracle.model_generator(oracle.MODEL_BD, [5.0, 1.0], [30])
    rho0 = synth.random_prob(30, 1)
    got, info = krylov.krylov_expv(A, rho0, [0.0], kappa=20)
    assert np.array_equal(got[0], rho0) and info["steps"] == 0
    Z = oracle.CSR.from_arrays([0, 1, 2], [0, 1], [0.0, 0.0])
    got, info = krylov.krylov_expv(Z, [0.25, 0.75], [3.0])
    assert np.array_equal(got[0], [0.25, 0.75])
