"""Pins for the oracle's generators of the paper's second and third models
(two-state birth-death, Sec. 3.1.2 / Eq. 2S_chem; autoregulatory gene network,
Sec. 3.1.3 / Eq. STS_chem), independent of the index arithmetic they use:

* a brute-force enumeration of the reaction network (stoichiometry vectors and
  propensities on a dict of states) gives the same generator on small grids;
* the gene state of the two-state model is a two-state chain: its marginal has
  the closed form a + (p0 - a) e^{-(l_act + l_ina) t};
* the mean R count solves dE/dt = beta P_act(t) - gamma E (closed form);
* with switching off, R is an immigration-death process (Poisson marginal)
  and, in the autoregulatory model, E[n_P] solves the linear moment ODE.
"""
import math

import numpy as np
import pytest
from scipy.stats import poisson

import oracle
from paper_2312_05647_amd import synth


def brute_generator(reactions, states, index):
    """reactions: list of (stoichiometry dict-free function, propensity);
    states: list of tuples; index: tuple -> linear index.  Off-grid moves are
    dropped (conservative).  Returns the dense generator."""
    N = len(states)
    A = np.zeros((N, N))
    for x in states:
        n = index[x]
        for move, prop in reactions:
            y, rate = move(x), prop(x)
            if rate == 0.0 or y not in index:
                continue
            A[n, index[y]] += rate
            A[n, n] -= rate
    return A


def same_generator(got, ref):
    """Off-diagonal rates identical; diagonals (sums of the exits, in another
    order) equal to rounding."""
    off = ~np.eye(len(ref), dtype=bool)
    assert np.array_equal(got[off], ref[off])
    assert np.abs(np.diag(got) - np.diag(ref)).max() <= 1e-13 * max(1.0, np.abs(np.diag(ref)).max())


def test_two_state_matches_reaction_enumeration():
    beta, gamma, lact, lina = 3.0, 0.7, 2.0, 1.0
    NR = 6
    states = [(r, s) for s in range(2) for r in range(NR)]
    index = {x: x[0] + NR * x[1] for x in states}
    reactions = [
        (lambda x: (x[0] + 1, x[1]), lambda x: beta if x[1] == 0 else 0.0),      # act -> R + act
        (lambda x: (x[0] - 1, x[1]), lambda x: gamma * x[0]),                    # R -> 0
        (lambda x: (x[0], 1), lambda x: lina if x[1] == 0 else 0.0),             # act -> ina
        (lambda x: (x[0], 0), lambda x: lact if x[1] == 1 else 0.0),             # ina -> act
    ]
    ref = brute_generator(reactions, states, index)
    got = oracle.model_generator(oracle.MODEL_TWOSTATE, [beta, gamma, lact, lina], [NR]).dense()
    same_generator(got, ref)


def test_autoreg_matches_reaction_enumeration():
    bR, bP, gR, gP, lact, lina = 2.5, 0.4, 1.0, 0.3, 0.1, 0.05
    NR, NP = 4, 5
    states = [(r, p, s) for s in range(2) for p in range(NP) for r in range(NR)]
    index = {x: x[0] + NR * x[1] + NR * NP * x[2] for x in states}
    reactions = [
        (lambda x: (x[0] + 1, x[1], x[2]), lambda x: bR if x[2] == 0 else 0.0),         # act -> R + act
        (lambda x: (x[0], x[1] + 1, x[2]), lambda x: bP * x[0]),                        # R -> R + P
        (lambda x: (x[0], x[1] - 1, 1), lambda x: lina * x[1] if x[2] == 0 else 0.0),   # act + P -> ina
        (lambda x: (x[0], x[1] + 1, 0), lambda x: lact if x[2] == 1 else 0.0),          # ina -> act + P
        (lambda x: (x[0] - 1, x[1], x[2]), lambda x: gR * x[0]),                        # R -> 0
        (lambda x: (x[0], x[1] - 1, x[2]), lambda x: gP * x[1]),                        # P -> 0
    ]
    ref = brute_generator(reactions, states, index)
    got = oracle.model_generator(oracle.MODEL_AUTOREG, [bR, bP, gR, gP, lact, lina], [NR, NP]).dense()
    same_generator(got, ref)
    assert np.abs(got.sum(axis=1)).max() < 1e-12


def test_leaky_rows_lose_only_the_capped_moves():
    A = oracle.model_generator(oracle.MODEL_AUTOREG, [2.5, 0.4, 1.0, 0.3, 0.1, 0.05], [4, 5], leaky=True).dense()
    rs = A.sum(axis=1)
    assert (rs <= 1e-15).all() and (rs < -1e-12).any()


def two_state_case(t, NR=160, beta=60.0, gamma=1.0, lact=2.0, lina=1.0, start_active=True):
    A = oracle.model_generator(oracle.MODEL_TWOSTATE, [beta, gamma, lact, lina], [NR])
    rho0 = synth.delta(2 * NR, 0 if start_active else NR)
    out, _ = oracle.expv(A, rho0, t, eps_right=1e-15)
    return out.reshape(2, NR)


@pytest.mark.parametrize("t", [0.2, 1.0, 4.0])
def test_two_state_gene_marginal_and_mean(t):
    beta, gamma, lact, lina = 60.0, 1.0, 2.0, 1.0
    P = two_state_case(t, beta=beta, gamma=gamma, lact=lact, lina=lina)
    lam = lact + lina
    a = lact / lam
    p_act = a + (1.0 - a) * math.exp(-lam * t)
    assert abs(P[0].sum() - p_act) < 1e-12
    mean = (P.sum(axis=0) * np.arange(P.shape[1])).sum()
    exact = beta * (a * (1 - math.exp(-gamma * t)) / gamma
                    + (1.0 - a) * (math.exp(-lam * t) - math.exp(-gamma * t)) / (gamma - lam))
    assert abs(mean - exact) < 1e-9 * exact


def test_two_state_without_switching_is_birth_death():
    P = two_state_case(1.5, lact=0.0, lina=0.0)
    assert P[1].sum() == 0.0
    exact = poisson.pmf(np.arange(P.shape[1]), 60.0 * (1 - math.exp(-1.5)))
    assert np.abs(P[0] - exact).sum() < 1e-10


def test_autoreg_without_switching_moments():
    bR, bP, gR, gP = 6.0, 0.5, 1.0, 0.4
    NR, NP = 30, 60
    t = 2.0
    A = oracle.model_generator(oracle.MODEL_AUTOREG, [bR, bP, gR, gP, 0.0, 0.0], [NR, NP])
    out, _ = oracle.expv(A, synth.delta(2 * NR * NP), t, eps_right=1e-15)
    P = out.reshape(2, NP, NR)
    assert P[1].sum() == 0.0
    pr = P[0].sum(axis=0)
    assert np.abs(pr - poisson.pmf(np.arange(NR), bR / gR * (1 - math.exp(-gR * t)))).sum() < 1e-10
    mean_p = (P[0].sum(axis=1) * np.arange(NP)).sum()
    exact = bP * bR / gR * ((1 - math.exp(-gP * t)) / gP - (math.exp(-gR * t) - math.exp(-gP * t)) / (gP - gR))
    assert abs(mean_p - exact) < 1e-8 * exact


def test_marginal_loglik_closed_form():
    """Two-state model with switching off, started active: the R marginal is
    Poisson((beta/gamma)(1 - e^{-gamma t})) and summing over the gene state
    adds nothing."""
    NR, beta = 160, 60.0
    A = oracle.model_generator(oracle.MODEL_TWOSTATE, [beta, 1.0, 0.0, 0.0], [NR])
    T = [0.5, 2.0]
    groups = [(0, [30, 30 + NR], 2), (1, [51, 51 + NR], 1), (1, [70, 70 + NR], 3)]
    got = oracle.loglik_marginal(A, synth.delta(2 * NR), T, groups, eps_right=1e-15)
    mean = [beta * (1 - math.exp(-t)) for t in T]
    ref = 2 * poisson.logpmf(30, mean[0]) + poisson.logpmf(51, mean[1]) + 3 * poisson.logpmf(70, mean[1])
    assert abs(got - ref) < 1e-9
