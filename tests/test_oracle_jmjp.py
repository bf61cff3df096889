"""Pins for the J-MJP oracle (Method #2: the state probabilities given the
jump counts, and the jump-count conditional), independent of its code:

* the Poisson(Omega T) mixture over k of (rho(0) B^k)_s is the transient
  distribution (uniformisation, Eq. ME_uniform): compared with scipy's
  matrix exponential;
* a pure birth chain (death rate 0) started at 0 moves up with probability
  beta/Omega per virtual jump until the cap, so (delta_0 B^k)_n is
  Binomial(n | k, beta/Omega);
* k = 0 gives rho(0); every B^k keeps the mass; a group of states sums;
* the jump-count conditional equals the brute-force product of the Poisson
  prior and the state probabilities, and its normaliser is rho(T)_s.
"""
import math

import numpy as np
import scipy.linalg as sl
from scipy.stats import binom, poisson

import oracle
from oracle import jmjp
from paper_2312_05647_amd import synth


def test_poisson_mixture_is_matrix_exponential():
    A = oracle.model_generator(oracle.MODEL_BD, [12.0, 0.8], [30])
    rho0 = synth.random_prob(30, 4)
    T = 0.7
    om = jmjp.omega(A)
    kmax = int(om * T + 12 * math.sqrt(om * T) + 30)
    ks = np.arange(kmax + 1)
    exact = rho0 @ sl.expm(A.dense() * T)
    for s in (0, 7, 19, 29):
        phi = jmjp.state_probs(A, rho0, [[s]] * len(ks), ks)
        mix = float(np.sum(poisson.pmf(ks, om * T) * phi))
        assert abs(mix - exact[s]) < 1e-13, (s, mix, exact[s])


def test_pure_birth_is_binomial():
    beta, N = 5.0, 60
    A = oracle.model_generator(oracle.MODEL_BD, [beta, 0.0], [N])
    om = jmjp.omega(A)
    assert om == 1.1 * beta
    for k in (0, 1, 5, 20, 45):
        phi = jmjp.state_probs(A, synth.delta(N), [[n] for n in range(N)], [k] * N)
        ref = binom.pmf(np.arange(N), k, beta / om)
        assert np.abs(phi - ref).max() < 1e-14, k


def test_k_zero_mass_and_groups():
    A = oracle.model_generator(oracle.MODEL_TWOSTATE, [30.0, 1.0, 2.0, 1.0], [40])
    rho0 = synth.random_prob(80, 9)
    assert np.array_equal(jmjp.state_probs(A, rho0, [[3], [50]], [0, 0]), rho0[[3, 50]])
    phi_all = jmjp.state_probs(A, rho0, [list(range(80))] * 4, [0, 3, 17, 60])
    assert np.abs(phi_all - 1.0).max() < 1e-13
    single = jmjp.state_probs(A, rho0, [[5], [45]], [11, 11])
    grouped = jmjp.state_probs(A, rho0, [[5, 45]], [11])
    assert abs(grouped[0] - single.sum()) < 1e-16
    # order of the observations does not matter
    ks = [9, 2, 9, 0, 5]
    a = jmjp.state_probs(A, rho0, [[i] for i in range(5)], ks)
    b = jmjp.state_probs(A, rho0, [[i] for i in range(5)][::-1], ks[::-1])
    assert np.array_equal(a, b[::-1])


def test_k_conditional_brute_force():
    A = oracle.model_generator(oracle.MODEL_BD, [6.0, 1.0], [25])
    rho0 = synth.delta(25)
    T, s = 1.2, 4
    om = jmjp.omega(A)
    kmax = 150                                   # Omega T = 39.6: the Poisson tail past 150 is ~1e-35
    cond = jmjp.k_conditional(A, rho0, [s], T, kmax)
    B = np.eye(25) + A.dense() / om
    brute = np.array([poisson.pmf(k, om * T) * np.linalg.matrix_power(B, k)[0, s] for k in range(kmax + 1)])
    assert np.abs(cond - brute / brute.sum()).max() < 1e-13
    # the normaliser is the transient probability (Poisson mean (beta/gamma)(1 - e^-T))
    assert abs(brute.sum() - poisson.pmf(s, 6.0 * (1 - math.exp(-T)))) < 1e-10


def test_log_joint():
    A = oracle.model_generator(oracle.MODEL_BD, [6.0, 1.0], [25])
    rho0 = synth.delta(25)
    om = jmjp.omega(A)
    groups, ks, T = [[2], [5], [3]], [4, 10, 7], [0.5, 1.0, 1.0]
    phi = jmjp.state_probs(A, rho0, groups, ks)
    ref = sum(poisson.logpmf(k, om * t) for k, t in zip(ks, T)) + np.log(phi).sum()
    assert abs(jmjp.log_joint(A, rho0, groups, ks, T) - ref) < 1e-12
    assert jmjp.log_joint(A, rho0, [[20]], [1], [1.0]) == -math.inf   # unreachable in one jump
