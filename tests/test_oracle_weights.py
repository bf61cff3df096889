"""Pins for the oracle's Poisson weights and jump-count rules.

The weights are the Poisson(k | Omega t) densities of Eq. ME_uniform; the
paper's cutoff is k* = W + 6 sqrt(W) (Sec. 2.2.3).  They are checked against
scipy.stats.poisson (a library routine the oracle does not call) and against
the error claim the paper prints for that cutoff.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.stats import poisson

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))

W_VALUES = [0.3, 2.0, 10.0, 87.5, 745.5, 1647.8, 2415.6, 8756.0]


@pytest.mark.parametrize("W", W_VALUES)
def test_weights_match_scipy_pmf(orc, W):
    K, _ = orc.pick_K(W, orc.K_TOL, 1e-15)
    w, total = orc.weights(W, K)
    k = np.arange(K + 1)
    ref = poisson.pmf(k, W)
    big = ref > 1e-250
    rel = np.abs(w[big] - ref[big]) / ref[big]
    # log-space formation: absolute log error ~ eps * (k log W) -> ~1e-12 relative
    assert rel.max() < 5e-11, rel.max()
    # each log w_k carries an absolute error of about eps * (W + k log W), a
    # common bias of the same order reaches the sum
    bound = 4 * 2.2e-16 * (W + (K + 1) * math.log(max(W, 1.0)))
    assert abs(total - poisson.cdf(K, W)) < max(bound, 1e-14)


@pytest.mark.parametrize("W", W_VALUES)
def test_weights_sum_to_one(orc, W):
    K, tail = orc.pick_K(W, orc.K_TOL, 1e-16)
    _, total = orc.weights(W, K)
    bound = 4 * 2.2e-16 * (W + (K + 1) * math.log(max(W, 1.0)))
    assert abs(total + tail - 1.0) < max(bound, 1e-14)


@pytest.mark.parametrize("W", W_VALUES)
@pytest.mark.parametrize("eps", [1e-6, 1e-10, 1e-13])
def test_tol_rule_is_smallest_K(orc, W, eps):
    K, tail = orc.pick_K(W, orc.K_TOL, eps)
    sf = poisson.sf(K, W)
    assert abs(tail - sf) <= 1e-10 * max(sf, 1e-300) + 1e-18
    assert sf <= eps * (1 + 1e-9)
    if K > 0:
        assert poisson.sf(K - 1, W) > eps * (1 - 1e-9)


def test_paper_rule_K_and_claimed_bound(orc):
    """Algorithm 2 loops while k <= k* with the increment first, so it makes
    floor(k*)+1 products; Sec. 2.2.3 claims the tail past k* is < 1e-5 when
    Omega t > 10."""
    mult = GOLDEN["kstar_sqrt_multiplier"]["value"]
    bound = GOLDEN["kstar_error_bound"]["value"]
    w_min = GOLDEN["kstar_error_bound"]["min_W_exclusive"]
    for W in np.concatenate([np.linspace(w_min + 1e-6, 50, 40), np.geomspace(50, 1e5, 40)]):
        K, tail = orc.pick_K(W, orc.K_PAPER, 0.0)
        kstar = W + mult * math.sqrt(W)
        assert K == math.floor(kstar) + 1
        # the paper's epsilon_{k*} sums k = 0..floor(k*)
        assert poisson.sf(math.floor(kstar), W) < bound
        assert tail < bound
        assert abs(tail - poisson.sf(K, W)) < 1e-12


def test_paper_rule_birth_death_count(orc):
    """Immigration-death with beta=500, gamma=1 on N=1000 (leaky exit rate of
    Sec. 3.1.1 is beta + gamma (N-1) = 1499; conservative is 1498): at t=1 the
    paper rule gives floor(W + 6 sqrt W) + 1 products."""
    W = 1.1 * 1498.0
    K, _ = orc.pick_K(W, orc.K_PAPER, 0.0)
    assert K == math.floor(W + 6 * math.sqrt(W)) + 1 == 1892


def test_logpmf_special_cases(orc):
    assert orc.poisson_logpmf(0, 0.0) == 0.0
    assert orc.poisson_logpmf(3, 0.0) == -math.inf
    assert abs(orc.poisson_logpmf(5, 3.0) - poisson.logpmf(5, 3.0)) < 1e-13
