"""Pins for the oracle's snapshot log-likelihood (Sec. 2.1.2): for the
birth-death process started at 0 the likelihood has the closed form
sum_i log Poisson(s_i; (beta/gamma)(1 - e^{-gamma T_i})), whose mean is the
mass-action formula the paper prints in the SI (Initialization)."""
import json
import math
import os

import numpy as np
from scipy.stats import poisson

from paper_2312_05647_amd import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_bd_loglik_closed_form(orc):
    d = GOLDEN["bd_data_design"]
    beta, gamma = float(d["betas"][0]), d["gamma"]
    T = np.linspace(d["t_lo"], d["t_hi"], d["n_times"])
    data = synth.gillespie_bd(beta, gamma, T, 40, seed=synth.SEED_DATA)
    N = max(2 * int(data[:, 1].max()), 150)        # 2x the largest count (Sec. 3.1.1)
    obs = synth.tally(data)                        # (time idx, count n, multiplicity)
    A = orc.model_generator(0, [beta, gamma], [N])
    ll = orc.loglik(A, synth.delta(N), T, obs)
    mean = beta / gamma * (1 - np.exp(-gamma * T))
    ref = sum(c * poisson.logpmf(s, mean[j]) for j, s, c in obs)
    assert abs(ll - ref) < 1e-9 * abs(ref)


def test_gillespie_bd_mean_matches_paper_formula():
    """The synthetic data itself: sample means per time against the SI's
    mass-action mean (beta/gamma)(1 - e^{-gamma T}) within 5 standard errors."""
    beta, gamma = 100.0, 1.0
    T = np.array([0.5, 2.0, 5.0])
    data = synth.gillespie_bd(beta, gamma, T, 400, seed=7)
    for j, t in enumerate(T):
        x = data[data[:, 0] == j, 1]
        mu = beta / gamma * (1 - math.exp(-gamma * t))
        assert abs(x.mean() - mu) < 5 * math.sqrt(mu / len(x))


def test_loglik_out_of_grid_is_minus_inf(orc):
    A = orc.model_generator(0, [5.0, 1.0], [20])
    obs = np.array([[0, 3, 1], [0, 25, 1]])
    assert orc.loglik(A, synth.delta(20), [1.0], obs) == -math.inf
