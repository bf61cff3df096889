"""GPU checks of the samplers: delayed acceptance reduces exactly to plain
Metropolis-Hastings when its screen is the exact posterior or a constant
(same random draws -> same paths), and both samplers recover a posterior
computed by quadrature for the two-rate birth-death model, whose likelihood
has a closed form (Poisson laws with mean (beta/gamma)(1 - e^{-gamma T}))."""
import sys

import numpy as np
import pytest
import torch
from scipy.stats import poisson

from paper_2312_05647_amd import mjp, sampler, synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def bd():
    beta, gamma = 50.0, 1.0
    T = np.linspace(0.5, 5.0, 10)
    data = synth.gillespie_bd(beta, gamma, T, 30, seed=synth.SEED_DATA)
    recs = np.array([[j, n, 0, c] for j, n, c in synth.tally(data)], np.int32)
    N = max(2 * int(data[:, 1].max()), 120)
    post = sampler.Posterior(mjp.MJP_MODEL_BD, T, recs, (N, 1), n_par=2)
    return post, T, recs, (beta, gamma)


def quadrature(T, recs, center, half=0.35, n=161):
    """Posterior mean and variance of (log beta, log gamma) on a grid."""
    a = np.linspace(center[0] - half, center[0] + half, n)
    b = np.linspace(center[1] - half, center[1] + half, n)
    A, Bg = np.meshgrid(a, b, indexing="ij")
    beta, gamma = np.exp(A), np.exp(Bg)
    lp = np.zeros_like(A)
    for j, x, _, c in recs:
        mean = beta / gamma * (1 - np.exp(-gamma * T[j]))
        lp += c * poisson.logpmf(x, mean)
    w = np.exp(lp - lp.max())
    w /= w.sum()
    m = np.array([(w * A).sum(), (w * Bg).sum()])
    v = np.array([(w * (A - m[0]) ** 2).sum(), (w * (Bg - m[1]) ** 2).sum()])
    return m, v


def test_da_with_exact_screen_equals_mh(bd):
    post, *_ = bd
    C, S = 64, 30
    gen = torch.Generator(device="cuda").manual_seed(1)
    psi0 = torch.log(torch.tensor([[50.0, 1.0]] * C, dtype=torch.float64, device="cuda"))
    Z = np.diag([4e-4, 4e-4])
    draws = sampler._draws(gen, S, C, 2)
    a, _ = sampler.run_mh(post, psi0, Z, S, None, draws=draws)
    b, st = sampler.run_da(post, post.logpost, psi0, Z, S, None, draws=draws)
    assert np.array_equal(a, b)
    assert st.accepted == st.stage1_accepted
    c, _ = sampler.run_da(post, lambda p: torch.zeros(p.shape[0], dtype=torch.float64, device="cuda"),
                          psi0, Z, S, None, draws=(draws[0], torch.flip(draws[1], dims=[2])))
    assert np.array_equal(a, c)   # constant screen: every proposal reaches the exact test


def test_both_samplers_match_quadrature(bd):
    post, T, recs, truth = bd
    C = 256
    gen = torch.Generator(device="cuda").manual_seed(2)
    psi0 = torch.log(torch.tensor([list(truth)] * C, dtype=torch.float64, device="cuda"))
    Z, psi = sampler.adapt_covariance(post, psi0, gen, rounds=4, steps=30)
    mq, vq = quadrature(T, recs, np.log(truth))
    # surrogate trained on exact log-likelihoods around the pilot posterior
    g = synth.rng(3)
    pts = g.multivariate_normal(mq, 9 * np.diag(vq), size=8192)
    ll = post.loglik(torch.as_tensor(pts, device="cuda")).cpu().numpy()
    screen, losses, _ = sampler.train_surrogate(pts, ll, epochs=60, batch=1024, seed=4)
    try:
        say(f"    surrogate loss {losses[0]:.3f} -> {losses[-1]:.5f}")
        for name, run in (("mh", lambda: sampler.run_mh(post, psi, Z, 300, gen)),
                          ("da", lambda: sampler.run_da(post, screen, psi, Z, 300, gen))):
            s, st = run()
            e = sampler.ess(s)
            flat = s.reshape(-1, 2)
            m, v = flat.mean(0), flat.var(0)
            mcse = np.sqrt(v / e)
            say(f"    {name}: mean {m} (quad {mq}) mcse {mcse}, var {v} (quad {vq}), ess {e}, exact {st.exact_evals}")
            assert np.all(np.abs(m - mq) < 4 * mcse + 1e-4 * np.abs(mq)), name
            assert np.all(np.abs(v - vq) < 0.25 * vq), name
            if name == "da":
                assert st.exact_evals < 0.8 * 300 * C
    finally:
        mjp.mjp_surrogate_destroy(screen.h)
