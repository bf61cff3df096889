"""Log-likelihoods of items too large for one workgroup's LDS (S1*S2 above
40,000 states): clusters of workgroups of one cooperative launch, each
owning a contiguous range of states and exchanging the boundary rows with
its neighbours every four jumps (a halo three rows deep recomputed by each
workgroup), or every jump, through the C ABI.

Against the FP64 oracle's independent per-time solves (Sec. 2.1.2) with the
log-likelihood bar of the batched path, |l_gpu - l_oracle| <=
sum_i c_i (2e-6 + 2e-9 / p_i) (FP32 products and accumulation, the 2.5e-10
Poisson cuts), on items just above the LDS capacity, well above it, at the
cluster's capacity (131,072 states, S1 = 1024), a birth-death item, and
mixed in one batch with small items (which the one-workgroup kernel runs);
an item beyond the clusters' capacity gets -inf with a flag.
"""
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


def run(model, theta, dims, T, recs, x0=(0, 0), opts=None):
    B = len(theta)
    th = torch.as_tensor(np.asarray(theta, np.float64), device="cuda").contiguous()
    dm = torch.as_tensor(np.asarray(dims, np.int32), device="cuda").contiguous()
    out = torch.empty(B, dtype=torch.float64, device="cuda")
    info = torch.zeros(B * ctypes.sizeof(mjp.mjp_info), dtype=torch.uint8, device="cuda")
    mjp.mjp_loglik(model, th, dm, mjp.make_obs(T, recs, x0), out, opts=opts, info=info)
    torch.cuda.synchronize()
    raw = info.cpu().numpy().tobytes()
    sz = ctypes.sizeof(mjp.mjp_info)
    return out.cpu().numpy(), [mjp.mjp_info.from_buffer_copy(raw[i * sz:(i + 1) * sz]) for i in range(B)]


def oracle(orc, model, theta, dims, T, recs):
    S1, S2 = int(dims[0]), int(dims[1])
    A = orc.model_generator(model, theta, [S1, S2] if model == orc.MODEL_CASCADE2 else [S1])
    n = S1 * S2
    rho = orc.expv_times(A, synth.delta(n), T)
    p = np.array([rho[j, x1 + S1 * x2] for j, x1, x2, _ in recs])
    c = recs[:, 3].astype(np.float64)
    ll = float((c * np.log(np.maximum(p, 1e-300))).sum())
    tol = float((c * (2e-6 + 2e-9 / np.maximum(p, 1e-300))).sum())
    return ll, tol, float(p.min())


def test_cluster_config():
    cfg = mjp.mjp_loglik_cluster_config()
    say(f"[gpu] cluster config {cfg}")
    assert cfg["clusters"] >= 1 and cfg["max_states"] >= 90000


def test_cluster_items_vs_oracle(orc):
    theta_star = [60.0, 1.0, 0.5, 0.5]
    T = np.array([0.4, 1.0, 2.0])
    data = synth.gillespie_cascade2(theta_star, T, 25, seed=synth.SEED_DATA)
    recs = synth.cascade_records(data)
    assert recs[:, 1].max() < 128 and recs[:, 2].max() < 128
    g = synth.rng(91)
    #            just above   well above  capacity     small (cell kernel)   beyond capacity
    grids = [(210, 200), (300, 300), (1024, 128), (130, 140), (90, 60), (400, 400)]
    theta = np.asarray(theta_star) * np.exp(g.uniform(-0.1, 0.1, size=(len(grids), 4)))
    got, info = run(mjp.MJP_MODEL_CASCADE2, theta, grids, T, recs)
    for b, S in enumerate(grids):
        n = S[0] * S[1]
        if n > 131072:
            say(f"    {S}: {got[b]} flags {info[b].flags}")
            assert got[b] == -np.inf and info[b].flags & mjp.MJP_FLAG_OUT_OF_GRID
            continue
        ll, tol, pmin = oracle(orc, orc.MODEL_CASCADE2, theta[b], S, T, recs)
        say(f"    {S} ({n} states): l {got[b]:.6f} oracle {ll:.6f} diff {abs(got[b] - ll):.2e} tol {tol:.2e} "
            f"p_min {pmin:.1e} mass {info[b].mass_out:.9f} K {info[b].K}")
        assert pmin > 1e-12 and np.isfinite(got[b])
        assert abs(got[b] - ll) <= tol, (S, got[b], ll, tol)
        assert abs(info[b].mass_out - 1.0) < 1e-5


def test_cluster_birth_death(orc):
    """Birth-death on 50,000 states (one state of reach), against the oracle
    and the closed form Poisson((beta/gamma)(1 - e^{-gamma T}))."""
    beta, gamma, N = 300.0, 1.0, 50000
    T = np.array([0.5, 1.5])
    data = synth.gillespie_bd(beta, gamma, T, 30, seed=synth.SEED_DATA)
    recs = np.array([[j, n, 0, c] for j, n, c in synth.tally(data)], np.int32)
    got, info = run(mjp.MJP_MODEL_BD, [[beta, gamma, 0.0, 0.0]], [(N, 1)], T, recs)
    ll, tol, pmin = oracle(orc, orc.MODEL_BD, [beta, gamma], (N, 1), T, recs)
    say(f"    birth-death N={N}: l {got[0]:.6f} oracle {ll:.6f} diff {abs(got[0] - ll):.2e} tol {tol:.2e}")
    assert abs(got[0] - ll) <= tol


def test_cluster_batch_repeatable():
    """Two calls give the same bits (the sums over a cluster's workgroups are
    added in rank order), and a batch with several large items per cluster
    (more items than clusters) matches item-by-item calls."""
    theta_star = [60.0, 1.0, 0.5, 0.5]
    T = np.array([0.4, 1.0])
    data = synth.gillespie_cascade2(theta_star, T, 10, seed=synth.SEED_DATA)
    recs = synth.cascade_records(data)
    g = synth.rng(92)
    B = 150
    theta = np.asarray(theta_star) * np.exp(g.uniform(-0.2, 0.2, size=(B, 4)))
    dims = np.array([(210 + (b % 7) * 10, 200 + (b % 5) * 10) for b in range(B)], np.int32)
    a, _ = run(mjp.MJP_MODEL_CASCADE2, theta, dims, T, recs)
    b2, _ = run(mjp.MJP_MODEL_CASCADE2, theta, dims, T, recs)
    assert np.isfinite(a).all() and np.array_equal(a, b2)
    for i in (0, 77, 149):
        one, _ = run(mjp.MJP_MODEL_CASCADE2, theta[i:i + 1], dims[i:i + 1], T, recs)
        assert one[0] == a[i], (i, one[0], a[i])


@pytest.mark.parametrize("renorm", [32, 0])
def test_cluster_four_jumps_bit_identical(renorm):
    """Four jumps per exchange (the halo states recomputed with the owner's
    cell update) against one jump per exchange (opts.variant
    MJP_VARIANT_PERSISTENT_ONEJUMP), bit for bit: cascade items from just
    above one workgroup's capacity to 300 x 300 and a wide one (S1 = 500),
    each with its own jump count (a last round of 1 to 4 jumps), with and
    without renormalisation."""
    theta_star = [60.0, 1.0, 0.5, 0.5]
    T = np.array([0.37, 1.0, 1.91])
    data = synth.gillespie_cascade2(theta_star, T, 12, seed=synth.SEED_DATA)
    recs = synth.cascade_records(data)
    g = synth.rng(93)
    grids = np.array([(210, 200), (300, 300), (500, 120), (256, 260), (233, 190)], np.int32)
    theta = np.asarray(theta_star) * np.exp(g.uniform(-0.15, 0.15, size=(len(grids), 4)))
    res = []
    for var in (mjp.MJP_VARIANT_AUTO, mjp.MJP_VARIANT_PERSISTENT_ONEJUMP):
        got, info = run(mjp.MJP_MODEL_CASCADE2, theta, grids, T, recs,
                        opts=mjp.mjp_opts_default(variant=var, renorm_every=renorm))
        res.append((got, [i.K for i in info], [i.mass_out for i in info]))
    say(f"    renorm {renorm}: K {res[0][1]} l {res[0][0]}")
    assert np.isfinite(res[0][0]).all()
    assert np.array_equal(res[0][0], res[1][0]) and res[0][2] == res[1][2]
