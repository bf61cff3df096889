"""The column kernel of the batched log-likelihood (cascade items: each lane
keeps one column segment of the grid in registers, neighbours by cross-lane
moves) through the C ABI.

* Against the FP64 oracle's independent per-time solves (Sec. 2.1.2) on grids
  that cover every register template, segments that wrap inside a wave,
  partial last segments, and grids too large for the column kernel (which
  fall back to the cell kernel).  Both sides use the paper's jump count
  K = floor(W + 6 sqrt W) + 1 and L = 0, so their truncation is identical and
  only the FP32 arithmetic differs.  Every jump forms each entry from nine
  rounded operations; the diagonal enters as x - (exit terms) x, which can
  amplify a rounding by (1 + e) / (1 - e) <= 21 (e <= 1/1.1 the exit
  probability), and the errors of the K jumps add like a random walk, so each
  observed probability carries a relative error <= 21 * 9 u sqrt(K) ~ 1e-5
  at K ~ 1500: bar |l_gpu - l_oracle| <= sum_i c_i 5e-5, compared for every
  item whose smallest observed probability exceeds 1e-30 (FP32's normal
  range ends at 1.2e-38).
* Against the cell kernel (mjp_loglik_set_kernel) on the same inputs, with
  twice that bar.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2312_05647_amd import mjp, synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

THETA_STAR = [12.0, 1.0, 0.6, 0.5]
# (S1, S2): column templates 8 (several with wave-crossing segment wraps),
# 24, 40, 50 (the 200-row columns of the batched workload's largest grids),
# 56 and 64 (one segment per column), and grids whose mirror exceeds the
# column kernel's LDS (cell kernel fallback)
GRIDS = [(40, 40), (41, 47), (63, 63), (45, 130), (60, 90), (110, 150), (160, 200), (200, 200),
         (199, 197), (700, 55), (500, 60), (130, 300), (170, 235)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def data():
    T = np.array([0.5, 1.5, 3.0])
    d = synth.gillespie_cascade2(THETA_STAR, T, 20, seed=synth.SEED_DATA)
    recs = synth.cascade_records(d)
    assert recs[:, 1].max() < 40 and recs[:, 2].max() < 40
    return T, recs


def run(theta, dims, T, recs, kernel, flags=False, **opts):
    mjp.mjp_loglik_set_kernel(1, kernel)
    try:
        B = len(theta)
        th = torch.as_tensor(np.asarray(theta, np.float64), device="cuda").contiguous()
        dm = torch.as_tensor(np.asarray(dims, np.int32), device="cuda").contiguous()
        out = torch.empty(B, dtype=torch.float64, device="cuda")
        sz = ctypes.sizeof(mjp.mjp_info)
        info = torch.zeros(B * sz, dtype=torch.uint8, device="cuda") if flags else None
        mjp.mjp_loglik(1, th, dm, mjp.make_obs(T, recs, (0, 0)), out, mjp.mjp_opts_default(**opts), info=info)
        torch.cuda.synchronize()
        if not flags:
            return out.cpu().numpy()
        raw = info.cpu().numpy().tobytes()
        fl = np.array([mjp.mjp_info.from_buffer_copy(raw[i * sz:(i + 1) * sz]).flags for i in range(B)])
        return out.cpu().numpy(), fl
    finally:
        mjp.mjp_loglik_set_kernel(1, mjp.MJP_LL_KERNEL_AUTO)


def oracle_item(orc, theta, dims, T, recs):
    S1, S2 = int(dims[0]), int(dims[1])
    A = orc.model_generator(orc.MODEL_CASCADE2, theta, [S1, S2])
    rho = orc.expv_times(A, synth.delta(S1 * S2), T, k_rule=orc.K_PAPER)
    p = np.array([rho[j, x1 + S1 * x2] for j, x1, x2, _ in recs])
    c = recs[:, 3].astype(np.float64)
    return float((c * np.log(np.maximum(p, 1e-300))).sum()), float(p.min()), float(c.sum())


def test_column_kernel_vs_oracle(orc, data):
    T, recs = data
    g = synth.rng(77)
    # per grid: a draw near theta* and two a decade away (small observed probabilities)
    theta, dims = [], []
    for S in GRIDS:
        for spread in (0.1, 1.0, 1.2):
            theta.append(np.asarray(THETA_STAR) * np.exp(g.uniform(-spread, spread, size=4)))
            dims.append(S)
    theta, dims = np.array(theta), np.array(dims, np.int32)
    got = run(theta, dims, T, recs, mjp.MJP_LL_KERNEL_AUTO, k_rule=mjp.MJP_K_PAPER)
    small = 0
    for b in range(len(theta)):
        ll, pmin, csum = oracle_item(orc, theta[b], dims[b], T, recs)
        bar = csum * 5e-5
        say(f"    {tuple(dims[b])}: l {got[b]:.6f} oracle {ll:.6f} diff {abs(got[b] - ll):.2e} bar {bar:.2e} "
            f"p_min {pmin:.1e}")
        if pmin <= 1e-30:
            continue
        small += pmin < 1e-12
        assert np.isfinite(got[b]) and abs(got[b] - ll) <= bar, (b, dims[b], got[b], ll)
    say(f"[gpu] column kernel: {small} items compared with p_min in (1e-30, 1e-12)")
    assert small >= 3


def test_column_kernel_vs_cell_kernel(data):
    T, recs = data
    g = synth.rng(78)
    theta = np.asarray(THETA_STAR) * np.exp(g.uniform(-0.3, 0.3, size=(len(GRIDS) * 4, 4)))
    dims = np.array([GRIDS[i % len(GRIDS)] for i in range(len(theta))], np.int32)
    a = run(theta, dims, T, recs, mjp.MJP_LL_KERNEL_AUTO)
    b = run(theta, dims, T, recs, mjp.MJP_LL_KERNEL_CELLS)
    bar = 2 * 5e-5 * recs[:, 3].sum()
    d = np.abs(a - b)
    say(f"[gpu] column vs cell kernel: max |diff| {d.max():.2e} (bar {bar:.2e})")
    assert np.isfinite(a).all() and (d <= bar).all()


def test_full_batch_column_vs_cells():
    """The 4096-draw batched workload (grids 148..200 per side): the column
    kernel and the cell kernel give the same finite/-inf pattern (up to
    items at the edge of FP32's range) and values within the bar above for
    every item whose observed probabilities all lie in FP32's normal range
    (neither kernel raises MJP_FLAG_SUBNORMAL_OBS).  Below 1.18e-38 a
    probability keeps fewer than 24 significant bits, so two kernels that
    round differently may differ there by more than the bar."""
    theta_star = [50.0, 1.0, 0.5, 0.5]
    T = synth.even_times(20, 0.5)
    d = synth.gillespie_cascade2(theta_star, T, 50, seed=synth.SEED_DATA)
    recs = synth.cascade_records(d)
    theta = synth.theta_draws(4096, theta_star, seed=synth.SEED_THETA)
    dims = synth.grid_dims(theta, (int(d[:, 1].max()), int(d[:, 2].max())))
    a, fla = run(theta, dims, T, recs, mjp.MJP_LL_KERNEL_AUTO, flags=True)
    b, flb = run(theta, dims, T, recs, mjp.MJP_LL_KERNEL_CELLS, flags=True)
    fa, fb = np.isfinite(a), np.isfinite(b)
    normal = ((fla | flb) & mjp.MJP_FLAG_SUBNORMAL_OBS) == 0
    both = fa & fb & normal
    say(f"[gpu] full batch: finite {fa.mean():.3f} (column) {fb.mean():.3f} (cells); "
        f"{(fa & fb & ~normal).sum()} finite items read a subnormal probability; "
        f"max |diff| over the other {both.sum()}: {np.abs(a[both] - b[both]).max():.2e}")
    assert (fa == fb).mean() > 0.99
    assert both.sum() > 0.6 * len(theta)
    bar = 2 * 5e-5 * recs[:, 3].sum()
    assert (np.abs(a[both] - b[both]) <= bar).all()
