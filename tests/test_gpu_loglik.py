"""GPU parity of the batched log-likelihood (mjp_loglik) against the FP64
oracle's independent per-time solves (Sec. 2.1.2), through the C ABI.

Bar: |l_gpu - l_oracle| <= sum_i c_i (2e-6 + 2e-9 / p_i) for every item:
FP32 products and accumulation give a relative error of a few 1e-7 per
probability, and the left and right Poisson cuts of 2.5e-10 each move at
most 1e-9 of absolute probability (lumped).  Items whose smallest oracle
probability is below 1e-12 are excluded from that comparison (checked for
-inf handling separately); test_cell_kernel_small_probabilities compares
items down to 1e-30 with identical truncation on both sides."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2312_05647_amd import mjp, synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_loglik(model, theta, dims, T, recs, x0=(0, 0), with_info=False, **opts):
    B = len(theta)
    th = torch.as_tensor(np.asarray(theta, np.float64).reshape(B, -1), device="cuda")
    if th.shape[1] < 4:
        th = torch.cat([th, torch.zeros(B, 4 - th.shape[1], dtype=th.dtype, device="cuda")], dim=1)
    dm = torch.as_tensor(np.asarray(dims, np.int32).reshape(B, 2), device="cuda")
    out = torch.empty(B, dtype=torch.float64, device="cuda")
    info = torch.zeros(B * ctypes.sizeof(mjp.mjp_info), dtype=torch.uint8, device="cuda") if with_info else None
    obs = mjp.make_obs(T, recs, x0)
    mjp.mjp_loglik(model, th.contiguous(), dm, obs, out, mjp.mjp_opts_default(**opts), info=info)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    if with_info:
        raw = info.cpu().numpy().tobytes()
        infos = [mjp.mjp_info.from_buffer_copy(raw[i * ctypes.sizeof(mjp.mjp_info):(i + 1) * ctypes.sizeof(mjp.mjp_info)])
                 for i in range(B)]
        return res, [i.as_dict() for i in infos]
    return res


def oracle_cascade(orc, theta, dims, T, recs, **kw):
    S1, S2 = int(dims[0]), int(dims[1])
    A = orc.model_generator(1, theta, [S1, S2])
    lin = []
    pmin = np.inf
    rho = orc.expv_times(A, synth.delta(S1 * S2), T, **kw)
    for j, x1, x2, c in recs:
        if x1 >= S1 or x2 >= S2:
            return -np.inf, 0.0, 0.0
        p = rho[j, x1 + S1 * x2]
        pmin = min(pmin, p)
        lin.append((j, x1 + S1 * x2, c))
    ll = orc.loglik(A, synth.delta(S1 * S2), T, np.array(lin), **kw)
    tol = sum(c * (2e-6 + 2e-9 / max(rho[j, s], 1e-300)) for j, s, c in lin)
    return ll, tol, pmin


@pytest.fixture(scope="module")
def small_case():
    theta_star = [12.0, 1.0, 0.6, 0.5]
    T = synth.even_times(4, 0.75)
    data = synth.gillespie_cascade2(theta_star, T, 25, seed=synth.SEED_DATA)
    recs = synth.cascade_records(data)
    theta = synth.theta_draws(48, theta_star, seed=synth.SEED_THETA)
    maxc = (int(data[:, 1].max()), int(data[:, 2].max()))
    dims = synth.grid_dims(theta, maxc, lo=20, hi=45)
    return theta, dims, T, recs


def test_small_batch_vs_oracle(orc, small_case):
    theta, dims, T, recs = small_case
    say(f"[gpu] loglik B={len(theta)} cascade, {len(recs)} records, {len(T)} times")
    got, info = run_loglik(1, theta, dims, T, recs, with_info=True)
    compared = 0
    for b in range(len(theta)):
        ll, tol, pmin = oracle_cascade(orc, theta[b], dims[b], T, recs)
        if ll == -np.inf:
            assert got[b] == -np.inf
            continue
        if pmin < 1e-12:
            continue
        assert abs(got[b] - ll) <= tol, (b, got[b], ll, tol)
        assert abs(info[b]["mass_out"] - 1.0) < 1e-5
        compared += 1
    assert compared >= len(theta) // 2


def test_birth_death_closed_form():
    """Immigration-death from 0: each record's probability is the Poisson
    pmf with mean (beta/gamma)(1 - e^{-gamma T}) (SI, Initialization)."""
    from scipy.stats import poisson
    T = np.linspace(0.5, 5.0, 10)
    data = synth.gillespie_bd(100.0, 1.0, T, 40, seed=3)
    recs = np.array([[j, n, 0, c] for j, n, c in synth.tally(data)])
    rng = synth.rng(5)
    theta = np.stack([100.0 * np.exp(rng.uniform(-0.3, 0.3, 16)), np.exp(rng.uniform(-0.3, 0.3, 16))], axis=1)
    dims = np.array([[400, 1]] * 16)
    say("[gpu] loglik birth-death closed form")
    got = run_loglik(0, theta, dims, T, recs)
    for b in range(16):
        beta, gamma = theta[b]
        mean = beta / gamma * (1 - np.exp(-gamma * T))
        p = np.array([poisson.pmf(n, mean[j]) for j, n, _, c in recs])
        ref = float(np.sum(recs[:, 3] * np.log(p)))
        tol = float(np.sum(recs[:, 3] * (2e-6 + 2e-9 / p)))
        assert abs(got[b] - ref) <= tol, (b, got[b], ref, tol)


def test_out_of_grid_and_over_cap(small_case):
    theta, dims, T, recs = small_case
    d = dims[:4].copy()
    d[1] = [3, 3]                      # observations fall outside this grid
    th = theta[:4].copy()
    th[2, 0] = 1e12                    # K far beyond the cap
    got, info = run_loglik(1, th, d, T, recs, with_info=True, k_cap=100000)
    assert got[1] == -np.inf and info[1]["flags"] & mjp.MJP_FLAG_OUT_OF_GRID
    assert got[2] == -np.inf and info[2]["flags"] & mjp.MJP_FLAG_K_LIMIT
    assert np.isfinite(got[0]) and np.isfinite(got[3])


def test_order_independent_and_deterministic(small_case):
    theta, dims, T, recs = small_case
    a = run_loglik(1, theta, dims, T, recs)
    b = run_loglik(1, theta, dims, T, recs)
    assert np.array_equal(a, b)
    perm = synth.rng(9).permutation(len(theta))
    c = run_loglik(1, theta[perm], dims[perm], T, recs)
    assert np.array_equal(c, a[perm])


def test_paper_rule(orc, small_case):
    theta, dims, T, recs = small_case
    got = run_loglik(1, theta[:6], dims[:6], T, recs, k_rule=mjp.MJP_K_PAPER)
    for b in range(6):
        ll, tol, pmin = oracle_cascade(orc, theta[b], dims[b], T, recs, k_rule=orc.K_PAPER)
        if np.isfinite(ll) and pmin > 1e-12:
            # the paper cutoff leaves a tail up to ~1e-6 on each side; both sides lump it the same way
            assert abs(got[b] - ll) <= tol + 1e-3, (b, got[b], ll)


def test_cell_kernel_small_probabilities(orc):
    """Items whose smallest observed probability lies in (1e-30, 1e-12),
    down to where FP32 still has its full precision: the paper's jump count
    K = floor(W + 6 sqrt W) + 1 and L = 0 on both sides, so the truncation is
    identical and only FP32 arithmetic differs.  Each entry of an iterate is
    formed from about nine rounded operations; the diagonal enters as
    x - (exit terms) x, which can amplify a rounding by (1 + e) / (1 - e) <= 21
    (e <= 1/1.1 the exit probability), and the K jumps' errors add like a
    random walk, so each observed probability carries a relative error
    <= 21 * 9 u sqrt(K) ~ 1e-5 at K ~ 1500: bar sum_i c_i 5e-5."""
    theta_star = [12.0, 1.0, 0.6, 0.5]
    T = np.array([0.5, 1.5, 3.0])
    d = synth.gillespie_cascade2(theta_star, T, 20, seed=synth.SEED_DATA)
    recs = synth.cascade_records(d)
    g = synth.rng(79)
    theta = np.array([np.asarray(theta_star) * np.exp(g.uniform(-1.2, 1.2, size=4)) for _ in range(24)])
    dims = np.array([(40 + 4 * (i % 5), 40 + 3 * (i % 7)) for i in range(len(theta))], np.int32)
    mjp.mjp_loglik_set_kernel(1, mjp.MJP_LL_KERNEL_CELLS)
    try:
        got = run_loglik(1, theta, dims, T, recs, k_rule=mjp.MJP_K_PAPER)
    finally:
        mjp.mjp_loglik_set_kernel(1, mjp.MJP_LL_KERNEL_AUTO)
    bar = 5e-5 * recs[:, 3].sum()
    small = 0
    for b in range(len(theta)):
        ll, _, pmin = oracle_cascade(orc, theta[b], dims[b], T, recs, k_rule=orc.K_PAPER)
        if not np.isfinite(ll) or pmin <= 1e-30:
            continue
        small += pmin < 1e-12
        assert abs(got[b] - ll) <= bar, (b, dims[b], got[b], ll, pmin)
    say(f"[gpu] cell kernel: {small} items compared with p_min in (1e-30, 1e-12)")
    assert small >= 3


@pytest.fixture(scope="module")
def full_case():
    """The batched workload: 4096 draws log-uniform over a decade around
    (50, 1, 0.5, 0.5), 20 collection times 0.5..10, 50 snapshots each,
    grids 50..200 per side."""
    theta_star = [50.0, 1.0, 0.5, 0.5]
    T = synth.even_times(20, 0.5)
    data = synth.gillespie_cascade2(theta_star, T, 50, seed=synth.SEED_DATA)
    recs = synth.cascade_records(data)
    theta = synth.theta_draws(4096, theta_star, seed=synth.SEED_THETA)
    maxc = (int(data[:, 1].max()), int(data[:, 2].max()))
    dims = synth.grid_dims(theta, maxc)
    return theta, dims, T, recs


def test_full_batch_sampled_items(orc, full_case):
    theta, dims, T, recs = full_case
    say(f"[gpu] loglik full batch B={len(theta)}, {len(recs)} records")
    got, info = run_loglik(1, theta, dims, T, recs, with_info=True)
    assert np.isfinite(got).mean() > 0.5
    # items the oracle can redo in seconds: the smallest grids and rates
    cost = np.array([i["K"] for i in info]) * dims[:, 0] * dims[:, 1]
    pick = list(np.argsort(cost)[:3]) + [int(np.argsort(cost)[len(cost) // 2])]
    for b in pick:
        say(f"    oracle item {b}: dims {dims[b]}, K {info[b]['K']}")
        ll, tol, pmin = oracle_cascade(orc, theta[b], dims[b], T, recs)
        if ll == -np.inf:
            assert got[b] == -np.inf
            continue
        if pmin < 1e-12:
            continue
        assert abs(got[b] - ll) <= tol, (b, got[b], ll, tol)


def test_graph_capture_replay(small_case):
    """mjp_loglik enqueues kernels only (after its first call uploads the
    observation tables), so it can be captured in a graph and replayed; every
    replay, with eager work and synchronisation between replays, must equal
    the eager result."""
    theta, dims, T, recs = small_case
    eager = run_loglik(1, theta, dims, T, recs)
    B = len(theta)
    th = torch.as_tensor(theta, device="cuda")
    dm = torch.as_tensor(np.asarray(dims, np.int32), device="cuda")
    out = torch.zeros(B, dtype=torch.float64, device="cuda")
    obs = mjp.make_obs(T, recs, (0, 0))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        mjp.mjp_loglik(1, th, dm, obs, out)   # same shapes: no growth inside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        mjp.mjp_loglik(1, th, dm, obs, out, stream=s)
    for rep in range(4):
        out.zero_()
        _ = (th * 2).sum()               # unrelated eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), rep


def _second_case():
    """Another observation set with the small case's batch shape: other
    rates, times and snapshots."""
    theta_star = [9.0, 0.8, 0.5, 0.7]
    T = synth.even_times(3, 0.6)
    data = synth.gillespie_cascade2(theta_star, T, 17, seed=synth.SEED_DATA + 7)
    recs = synth.cascade_records(data)
    return T, recs


def test_graph_keeps_its_observations(small_case):
    """A graph captured from a call keeps the records it was captured with:
    an eager call with another observation set between replays (the same
    number of items, so nothing grows) changes neither the replays nor its
    own result.  The replays run on the capturing stream, ordered after the
    eager call: a graph shares that stream's work tables, so it must not run
    concurrently with another call on the stream."""
    theta, dims, T, recs = small_case
    T2, recs2 = _second_case()
    eager_a = run_loglik(1, theta, dims, T, recs)
    eager_b = run_loglik(1, theta, dims, T2, recs2)
    assert not np.array_equal(eager_a, eager_b)
    B = len(theta)
    th = torch.as_tensor(theta, device="cuda")
    dm = torch.as_tensor(np.asarray(dims, np.int32), device="cuda")
    out = torch.zeros(B, dtype=torch.float64, device="cuda")
    out_b = torch.zeros(B, dtype=torch.float64, device="cuda")
    obs_a, obs_b = mjp.make_obs(T, recs, (0, 0)), mjp.make_obs(T2, recs2, (0, 0))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        mjp.mjp_loglik(1, th, dm, obs_a, out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        mjp.mjp_loglik(1, th, dm, obs_a, out, stream=s)
    for rep in range(3):
        out.zero_()
        out_b.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            mjp.mjp_loglik(1, th, dm, obs_b, out_b, stream=s)   # other records, same stream
            g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager_a), rep
        assert np.array_equal(out_b.cpu().numpy(), eager_b), rep


def test_two_streams_do_not_share_tables(small_case):
    """Calls on two streams, enqueued back to back without a
    synchronisation between them, each with its own observation set, give
    what each gives alone."""
    theta, dims, T, recs = small_case
    T2, recs2 = _second_case()
    eager_a = run_loglik(1, theta, dims, T, recs)
    eager_b = run_loglik(1, theta, dims, T2, recs2)
    B = len(theta)
    th = torch.as_tensor(theta, device="cuda")
    dm = torch.as_tensor(np.asarray(dims, np.int32), device="cuda")
    obs_a, obs_b = mjp.make_obs(T, recs, (0, 0)), mjp.make_obs(T2, recs2, (0, 0))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for rep in range(3):
        out_a = torch.zeros(B, dtype=torch.float64, device="cuda")
        out_b = torch.zeros(B, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        mjp.mjp_loglik(1, th, dm, obs_a, out_a, stream=s1)
        mjp.mjp_loglik(1, th, dm, obs_b, out_b, stream=s2)
        torch.cuda.synchronize()
        assert np.array_equal(out_a.cpu().numpy(), eager_a), rep
        assert np.array_equal(out_b.cpu().numpy(), eager_b), rep
