"""The device samplers (mjp_sampler_*) through the C ABI.

* The device generator equals the host one (and so the oracle's Philox).
* Delayed acceptance with a constant screen equals plain MH path for path
  (same seed, start and covariance), and both recover the posterior of the
  two-rate birth-death model computed by quadrature (closed-form
  likelihood: Poisson laws with mean (beta/gamma)(1 - e^{-gamma T})).
* A step captured in a graph and replayed (with eager work and
  synchronisation between replays) gives the chains of eager steps.
* A checkpoint (states, log-posteriors, counters) restored into a new
  sampler continues the chains exactly.
"""
import sys

import numpy as np
import pytest
import torch
from scipy.stats import poisson

from oracle import philox
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
    a = np.linspace(center[0] - half, center[0] + half, n)
    b = np.linspace(center[1] - half, center[1] + half, n)
    A, Bg = np.meshgrid(a, b, indexing="ij")
    beta, gamma = np.exp(A), np.exp(Bg)
    lp = np.zeros_like(A)
    for j, x, _, c in recs:
        lp += c * poisson.logpmf(x, beta / gamma * (1 - np.exp(-gamma * T[j])))
    w = np.exp(lp - lp.max())
    w /= w.sum()
    m = np.array([(w * A).sum(), (w * Bg).sum()])
    v = np.array([(w * (A - m[0]) ** 2).sum(), (w * (Bg - m[1]) ** 2).sum()])
    return m, v


def zero_screen(d):
    """A surrogate whose output is exactly 0 (all parameters zero)."""
    h = mjp.mjp_surrogate_create(d, 64, 1, seed=1)
    mjp.mjp_surrogate_set_params(h, np.zeros(mjp.mjp_surrogate_num_params(h), np.float32))
    return sampler.SurrogateScreen(h, np.zeros(d), np.ones(d), 0.0, 1.0)


def test_device_generator_matches_host_and_oracle():
    out = torch.zeros(4 * 1000, dtype=torch.int32, device="cuda")
    key = 0x0123456789ABCDEF
    mjp.mjp_philox_fill(key, 7, 11, 3, out)
    got = out.cpu().numpy().view(np.uint32).reshape(-1, 4)
    for i in (0, 1, 2, 500, 999):
        ref = philox.philox4x32([i, 7, 11, 3], [key & 0xFFFFFFFF, key >> 32])
        assert list(map(int, got[i])) == ref, i
        assert list(map(int, mjp.mjp_philox4x32_10([i, 7, 11, 3], [key & 0xFFFFFFFF, key >> 32]))) == ref


def test_constant_screen_delayed_acceptance_equals_mh(bd):
    post, *_ = bd
    C, S = 128, 40
    psi0 = torch.log(torch.tensor([[50.0, 1.0]] * C, dtype=torch.float64, device="cuda"))
    psi0 += 0.01 * torch.randn(psi0.shape, generator=torch.Generator(device="cuda").manual_seed(3),
                               device="cuda", dtype=torch.float64)
    Z = np.diag([4e-4, 4e-4])
    a, sa = sampler.run_device(post, psi0, Z, S, seed=77)
    screen = zero_screen(2)
    try:
        b, sb = sampler.run_device(post, psi0, Z, S, seed=77, screen=screen)
    finally:
        mjp.mjp_surrogate_destroy(screen.h)
    say(f"    MH accepted {sa.accepted}, DA accepted {sb.accepted} (stage 1 {sb.stage1_accepted} of {C * S})")
    assert np.array_equal(a, b)
    assert sa.accepted == sb.accepted and sb.stage1_accepted == C * S
    assert 0.1 < sa.accepted / (C * S) < 0.9
    # a different seed gives different chains
    c, _ = sampler.run_device(post, psi0, Z, S, seed=78)
    assert not np.array_equal(a, c)


def test_device_samplers_match_quadrature(bd):
    post, T, recs, truth = bd
    C = 256
    gen = torch.Generator(device="cuda").manual_seed(2)
    psi0 = torch.log(torch.tensor([list(truth)] * C, dtype=torch.float64, device="cuda"))
    Z, psi = sampler.adapt_covariance(post, psi0, gen, rounds=4, steps=30)
    mq, vq = quadrature(T, recs, np.log(truth))
    g = synth.rng(3)
    pts = g.multivariate_normal(mq, 9 * np.diag(vq), size=8192)
    ll = post.loglik(torch.as_tensor(pts, device="cuda")).cpu().numpy()
    screen, losses, _ = sampler.train_surrogate(pts, ll, epochs=60, batch=1024, seed=4)
    try:
        for name, scr in (("mh", None), ("da", screen)):
            s, st = sampler.run_device(post, psi, Z, 300, seed=5, screen=scr)
            e = sampler.ess(s)
            flat = s.reshape(-1, 2)
            m, v = flat.mean(0), flat.var(0)
            mcse = np.sqrt(v / e)
            say(f"    device {name}: mean {m} (quad {mq}) mcse {mcse}, var {v} (quad {vq}), ess {e}, "
                f"exact {st.exact_evals}, {st.seconds:.2f} s")
            assert np.all(np.abs(m - mq) < 4 * mcse + 1e-4 * np.abs(mq)), name
            assert np.all(np.abs(v - vq) < 0.25 * vq), name
            if name == "da":
                assert st.exact_evals < 0.8 * 300 * C
    finally:
        mjp.mjp_surrogate_destroy(screen.h)


def test_graph_replay_equals_eager_steps(bd):
    post, *_ = bd
    C, N = 64, 6
    psi0 = torch.log(torch.tensor([[50.0, 1.0]] * C, dtype=torch.float64, device="cuda"))
    Z = np.diag([4e-4, 4e-4])
    screen = zero_screen(2)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    try:
        for scr in (None, screen):
            ref = sampler.DeviceChains(post, C, 9, Z, scr)
            gr = sampler.DeviceChains(post, C, 9, Z, scr)
            try:
                ring_ref = torch.zeros((N + 1, C, 2), dtype=torch.float64, device="cuda")
                ring_gr = torch.zeros_like(ring_ref)
                with torch.cuda.stream(s):
                    ref.init(psi0, stream=s)
                    ref.run(N + 1, ring_ref, stream=s)
                    gr.init(psi0, stream=s)
                    gr.run(1, ring_gr, stream=s)  # eager first step on the capture stream
                torch.cuda.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=s):
                    gr.run(1, ring_gr, stream=s)
                for i in range(N):
                    g.replay()
                    torch.cuda.synchronize()
                    junk = torch.ones(1000, device="cuda") * (i + 1)  # eager work between replays
                    torch.cuda.synchronize()
                    assert float(junk.sum()) == 1000.0 * (i + 1)
                assert torch.equal(ring_ref, ring_gr), "screen" if scr else "mh"
                assert np.array_equal(ref.state()["psi"], gr.state()["psi"])
                assert list(gr.state()["counters"][:1]) == [N + 1]
            finally:
                ref.close()
                gr.close()
    finally:
        mjp.mjp_surrogate_destroy(screen.h)


def test_checkpoint_resume_continues_the_chains(bd):
    post, *_ = bd
    C, S = 96, 20
    psi0 = torch.log(torch.tensor([[50.0, 1.0]] * C, dtype=torch.float64, device="cuda"))
    Z = np.diag([4e-4, 4e-4])
    screen = zero_screen(2)
    try:
        for scr in (None, screen):
            full = sampler.DeviceChains(post, C, 21, Z, scr)
            part = sampler.DeviceChains(post, C, 21, Z, scr)
            try:
                a = torch.zeros((2 * S, C, 2), dtype=torch.float64, device="cuda")
                full.init(psi0)
                full.run(2 * S, a)
                b = torch.zeros_like(a)
                part.init(psi0)
                part.run(S, b)
                ck = part.state()
                part.close()
                part = sampler.DeviceChains(post, C, 21, Z, scr)
                part.set_state(ck)
                part.run(S, b)
                torch.cuda.synchronize()
                assert torch.equal(a, b)
                assert np.array_equal(full.state()["counters"], part.state()["counters"])
            finally:
                full.close()
                part.close()
    finally:
        mjp.mjp_surrogate_destroy(screen.h)


def test_device_poisson_draws_follow_the_law():
    """Chi-square of 200,000 device draws against the Poisson pmf, for means
    on both sides of the inversion / transformed-rejection switch."""
    from scipy.stats import chi2
    n = 200000
    for lam in (0.3, 3.0, 9.99, 10.0, 37.5, 500.0, 4000.0):
        lt = torch.full((n,), lam, dtype=torch.float64, device="cuda")
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        mjp.mjp_poisson_fill(99, int(lam * 100), lt, out)
        x = out.cpu().numpy()
        lo, hi = int(poisson.ppf(1e-4, lam)), int(poisson.ppf(1 - 1e-4, lam))
        edges = np.unique(np.linspace(lo, hi + 1, 40).astype(int))
        obs, _ = np.histogram(x, bins=np.concatenate([[-np.inf], edges[1:-1], [np.inf]]))
        cdf = poisson.cdf(edges[1:-1] - 1, lam)
        p = np.diff(np.concatenate([[0.0], cdf, [1.0]]))
        keep = p * n > 5
        stat = ((obs[keep] - n * p[keep]) ** 2 / (n * p[keep])).sum()
        dof = keep.sum() - 1
        say(f"    Poisson({lam}): mean {x.mean():.4f} var {x.var():.4f} chi2 {stat:.1f} dof {dof}")
        assert stat < chi2.ppf(1 - 1e-4, dof), lam
        assert abs(x.mean() - lam) < 6 * np.sqrt(lam / n)


def test_device_jmjp_matches_quadrature():
    """J-MJP Gibbs with every step on the device: the theta marginal of the
    birth-death posterior (10 times x 30 snapshots) against quadrature."""
    from paper_2312_05647_amd import jmjp
    beta, gamma = 50.0, 1.0
    T = np.linspace(0.5, 5.0, 10)
    data = synth.gillespie_bd(beta, gamma, T, 30, seed=synth.SEED_DATA)
    recs = np.array([[j, n, 0, c] for j, n, c in synth.tally(data)], np.int32)
    N = max(2 * int(data[:, 1].max()), 120)
    mq, vq = quadrature(T, recs, np.log([beta, gamma]))
    C, S = 256, 600
    g = synth.rng(12)
    psi0 = torch.as_tensor(g.multivariate_normal(mq, np.diag(vq), size=C), device="cuda")
    Z = np.diag(vq) * 2.38 ** 2 / 2
    post = jmjp.JumpPosterior(0, T, recs, (N, 1), n_par=2)
    s, st = jmjp.run_jmjp_device(post, psi0, Z, S, seed=31)
    e = sampler.ess(s)
    flat = s.reshape(-1, 2)
    m, v = flat.mean(0), flat.var(0)
    mcse = np.sqrt(v / e)
    say(f"    device jmjp: mean {m} (quad {mq}) mcse {mcse}, var {v} (quad {vq}), ess {e}, "
        f"theta acc {st.theta_accepted / (S * C):.3f}, k acc {st.k_accept_rate:.3f}, {st.seconds:.1f} s")
    assert np.all(np.abs(m - mq) < 4 * mcse + 1e-4 * np.abs(mq))
    assert np.all(np.abs(v - vq) < 0.3 * vq)
    assert 0.05 < st.k_accept_rate < 0.99  # the host Gibbs sampler measures 0.951 here
