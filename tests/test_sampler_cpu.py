"""Host-side checks of the sampler's post-processing: the autocorrelation
(the paper's Eq. autocorr) and the effective sample size, against an AR(1)
process whose integrated autocorrelation time is known in closed form:
tau = (1 + phi) / (1 - phi)."""
import numpy as np
import pytest

from paper_2312_05647_amd import sampler, synth


@pytest.mark.parametrize("phi", [0.0, 0.5, 0.9])
def test_ess_of_ar1(phi):
    g = synth.rng(4)
    S, C = 4000, 8
    x = np.zeros((S, C, 1))
    e = g.normal(size=(S, C))
    for t in range(1, S):
        x[t, :, 0] = phi * x[t - 1, :, 0] + e[t]
    tau = (1 + phi) / (1 - phi)
    got = sampler.ess(x)[0]
    assert abs(got - S * C / tau) < 0.2 * S * C / tau


def test_acf_basic():
    x = np.array([1.0, -1.0] * 50)
    rho = sampler.autocorrelation(x)
    assert rho[0] == pytest.approx(1.0)
    assert rho[1] == pytest.approx(-1.0)
    assert rho[2] == pytest.approx(1.0)
