"""Pins for the oracle's R-MJP expansion (Algorithm 2) against things other
than itself: the immigration-death closed form, scipy's dense expm, the
two-species moment equations, and invariants the mathematics fixes (mass,
Omega-invariance, the semigroup law, linearity, the truncation bound of the
lumped series)."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm
from scipy.stats import poisson

from paper_2312_05647_amd import synth


def random_generator(n, seed, dense=False, scale=5.0):
    import oracle
    rp, c, r = synth.random_rate_graph(n, seed, degree=3, scale=scale, dense=dense)
    return oracle.CSR.from_arrays(*synth.with_generator_diagonal(rp, c, r))


def test_bd_closed_form_small_workload(orc):
    """Immigration-death from 0 has law Poisson((lam/mu)(1 - e^{-mu t}));
    N = 1000, lam = 500, mu = 1, t = 1 (mean 316.06, far from the cutoff)."""
    A = orc.model_generator(0, [500.0, 1.0], [1000])
    out, info = orc.expv(A, synth.delta(1000), 1.0)
    exact = poisson.pmf(np.arange(1000), 500.0 * (1 - math.exp(-1.0)))
    assert np.abs(out - exact).sum() < 1e-10
    assert info["K"] > info["W"]


def test_bd_stationary_law(orc):
    """For large t the birth-death law tends to Poisson(beta/gamma) (Sec. 3.1.1)."""
    A = orc.model_generator(0, [60.0, 1.0], [200])
    out, _ = orc.expv(A, synth.delta(200, 5), 40.0)
    assert np.abs(out - poisson.pmf(np.arange(200), 60.0)).sum() < 1e-9


@pytest.mark.parametrize("n,seed", [(5, 1), (17, 2), (40, 3), (64, 4)])
def test_dense_expm_random_sparse(orc, n, seed):
    A = random_generator(n, seed)
    rho0 = synth.random_prob(n, seed + 100)
    t = 0.05 + 1.5 * synth.rng(seed + 200).uniform()
    out, info = orc.expv(A, rho0, t)
    exact = rho0 @ expm(A.dense() * t)
    assert np.abs(out - exact).sum() < 1e-11
    # the check can see a transposed operand: the column-vector product differs
    assert np.abs(expm(A.dense() * t) @ rho0 - exact).sum() > 1e-3


def test_dense_expm_dense_graph(orc):
    A = random_generator(20, 9, dense=True, scale=2.0)
    rho0 = synth.random_prob(20, 10)
    out, _ = orc.expv(A, rho0, 0.7)
    assert np.abs(out - rho0 @ expm(A.dense() * 0.7)).sum() < 1e-11


def _moment_ode(theta, t):
    k1, g1, k2, g2 = theta

    def f(_, y):
        m1, m2, c11, c12, c22 = y
        return [k1 - g1 * m1, k2 * m1 - g2 * m2, k1 + g1 * m1 - 2 * g1 * c11,
                k2 * c11 - (g1 + g2) * c12, k2 * m1 + g2 * m2 + 2 * k2 * c12 - 2 * g2 * c22]

    sol = solve_ivp(f, (0, t), [0.0] * 5, method="DOP853", rtol=1e-13, atol=1e-13)
    return sol.y[:, -1]


def test_cascade2_marginal_and_moments(orc):
    """Species 1 of the cascade is an independent immigration-death, so its
    marginal is Poisson((k1/g1)(1-e^{-g1 t})); the first and second moments of
    (n1, n2) follow the exact moment equations of a network with affine
    propensities."""
    theta = [20.0, 1.0, 0.5, 0.5]
    S1, S2, t = 60, 60, 2.0
    A = orc.model_generator(1, theta, [S1, S2])
    out, _ = orc.expv(A, synth.delta(S1 * S2), t)
    P = out.reshape(S2, S1)          # P[n2, n1]
    m1 = poisson.pmf(np.arange(S1), theta[0] / theta[1] * (1 - math.exp(-theta[1] * t)))
    assert np.abs(P.sum(0) - m1).sum() < 1e-11
    n1 = np.arange(S1)[None, :]
    n2 = np.arange(S2)[:, None]
    E1, E2 = (P * n1).sum(), (P * n2).sum()
    C11 = (P * n1 * n1).sum() - E1 ** 2
    C12 = (P * n1 * n2).sum() - E1 * E2
    C22 = (P * n2 * n2).sum() - E2 ** 2
    ref = _moment_ode(theta, t)
    got = np.array([E1, E2, C11, C12, C22])
    assert np.allclose(got, ref, rtol=1e-9, atol=1e-10), (got, ref)


def test_mass_with_and_without_lumping(orc):
    """Lumped (the last line of Algorithm 2): output mass = input mass.
    Without it the mass is sum_{k<=K} w_k = 1 - residual exactly."""
    A = orc.model_generator(1, [30.0, 1.0, 0.5, 0.5], [40, 40])
    rho0 = synth.random_prob(1600, 3)
    out, info = orc.expv(A, rho0, 1.0, eps_right=1e-6)
    assert abs(out.sum() - 1.0) < 1e-13
    out2, info2 = orc.expv(A, rho0, 1.0, eps_right=1e-6, lump=False)
    assert abs(out2.sum() - (1.0 - info2["residual"])) < 1e-13
    assert abs(info2["residual"] - info2["eps_right"]) < 1e-12
    assert 1e-7 < info2["residual"] <= 1e-6


@pytest.mark.parametrize("factor", [1.5, 2.0, 3.7])
def test_omega_invariance(orc, factor):
    """Omega may be any value above max|a_nn| (Eq. B_def); the exact result
    does not depend on it."""
    A = random_generator(30, 5)
    rho0 = synth.random_prob(30, 6)
    a, _ = orc.expv(A, rho0, 0.9, omega_factor=1.1)
    b, _ = orc.expv(A, rho0, 0.9, omega_factor=factor)
    assert np.abs(a - b).sum() < 1e-12


def test_semigroup(orc):
    A = orc.model_generator(1, [10.0, 1.0, 0.8, 0.6], [30, 25])
    rho0 = synth.delta(750)
    ab, _ = orc.expv(A, orc.expv(A, rho0, 0.4)[0], 1.1)
    c, _ = orc.expv(A, rho0, 1.5)
    assert np.abs(ab - c).sum() < 1e-12


def test_linearity(orc):
    A = random_generator(25, 7)
    r1, r2 = synth.random_prob(25, 1), synth.random_prob(25, 2)
    f = lambda r: orc.expv(A, r, 0.6)[0]
    assert np.abs(f(0.3 * r1 + 2.0 * r2) - (0.3 * f(r1) + 2.0 * f(r2))).sum() < 1e-12


def test_paper_rule_error_within_lumping_bound(orc):
    """With the paper's cutoff and the residual lumped onto the last iterate,
    the L1 error is at most 2 x (dropped tail): each dropped w_k rho_k is
    replaced by w_k rho_K and both have unit mass.  A small W makes the tail
    measurable."""
    A = orc.model_generator(0, [4.0, 1.0], [30])
    m = 4.0 + 28.0
    t = 12.0 / (1.1 * m)
    rho0 = synth.delta(30)
    out, info = orc.expv(A, rho0, t, k_rule=orc.K_PAPER)
    assert info["K"] == math.floor(12.0 + 6 * math.sqrt(12.0)) + 1
    exact = rho0 @ expm(A.dense() * t)
    err = np.abs(out - exact).sum()
    assert err <= 2 * info["eps_right"] + 1e-13
    assert err > 1e-3 * info["eps_right"]   # the truncation is really there
    # dropping the lumping line leaves exactly the tail mass missing
    out_nl, _ = orc.expv(A, rho0, t, k_rule=orc.K_PAPER, lump=False)
    assert abs((exact.sum() - out_nl.sum()) - info["eps_right"]) < 1e-13


def test_special_cases(orc):
    A = random_generator(10, 11)
    rho0 = synth.random_prob(10, 12)
    out, info = orc.expv(A, rho0, 0.0)
    assert np.array_equal(out, rho0) and info["K"] == 0
    Z = orc.CSR.from_arrays(np.arange(11, dtype=np.int64), np.arange(10, dtype=np.int32), np.zeros(10))
    out, _ = orc.expv(Z, rho0, 3.0)
    assert np.array_equal(out, rho0)
    with pytest.raises(ValueError):
        orc.expv(A, rho0, -1.0)
    with pytest.raises(ValueError):
        orc.expv(A, rho0, 1.0, omega_factor=1.0)


@pytest.mark.parametrize("seed", [21, 22])
def test_single_jump_vs_dense(orc, seed):
    A = random_generator(33, seed)
    x = synth.random_prob(33, seed + 1)
    D = A.dense()
    omega = 1.1 * np.abs(np.diag(D)).max()
    ref = x @ (np.eye(33) + D / omega)
    assert np.abs(orc.jump(A, x) - ref).max() < 1e-15


def test_nonnegative(orc):
    A = orc.model_generator(1, [50.0, 1.0, 0.5, 0.5], [80, 60])
    out, _ = orc.expv(A, synth.delta(4800), 3.0)
    assert (out >= 0).all()
