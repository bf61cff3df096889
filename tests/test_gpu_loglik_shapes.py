"""Launch shapes and the autotuner of the batched log-likelihood through the
C ABI: every shape against the FP64 oracle, items of all four size classes
in one batch, the tuner's report and choice, the record-capacity fallback,
and the class grouping of a batch too large to sort.

Bar against the oracle: the log-likelihood bar of the batched path,
|l_gpu - l_oracle| <= sum_i c_i (2e-6 + 2e-9 / p_i) (FP32 products and
accumulation, 2.5e-10 Poisson cuts).  One item's arithmetic does not depend
on the batch around it, so the same item under the same shape is compared
bit for bit.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2312_05647_amd import mjp, synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

GRIDS = [(40, 40), (60, 90), (110, 150), (160, 200)]     # 1600, 5400, 16500, 32000 states: classes 0..3


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def shape_class(n):
    lim = mjp.mjp_loglik_class_limits()
    return next(c for c, l in enumerate(lim) if n <= l)


@pytest.fixture(autouse=True)
def default_shapes():
    """The cell kernel (whose shapes these tests cover) for every cascade item."""
    mjp.mjp_loglik_set_kernel(1, mjp.MJP_LL_KERNEL_CELLS)
    mjp.mjp_loglik_set_shapes(1, [-1] * 4)
    yield
    mjp.mjp_loglik_set_shapes(1, [-1] * 4)
    mjp.mjp_loglik_set_kernel(1, mjp.MJP_LL_KERNEL_AUTO)


@pytest.fixture(scope="module")
def mixed():
    """16 cascade items, 4 per size class, rates around (12, 1, 0.6, 0.5)."""
    theta_star = [12.0, 1.0, 0.6, 0.5]
    T = np.array([0.5, 1.5, 3.0])
    data = synth.gillespie_cascade2(theta_star, T, 20, seed=synth.SEED_DATA)
    recs = synth.cascade_records(data)
    g = synth.rng(synth.SEED_THETA)                  # draws near theta*, so the data are likely
    theta = np.asarray(theta_star) * np.exp(g.uniform(-0.15, 0.15, size=(16, 4)))
    dims = np.array([GRIDS[i // 4] for i in range(16)], np.int32)
    assert recs[:, 1].max() < 40 and recs[:, 2].max() < 40
    return theta, dims, T, recs


def run(theta, dims, T, recs):
    B = len(theta)
    th = torch.as_tensor(np.asarray(theta, np.float64), device="cuda").contiguous()
    dm = torch.as_tensor(np.asarray(dims, np.int32), device="cuda").contiguous()
    out = torch.empty(B, dtype=torch.float64, device="cuda")
    mjp.mjp_loglik(1, th, dm, mjp.make_obs(T, recs), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.fixture(scope="module")
def oracle_values(orc, mixed):
    theta, dims, T, recs = mixed
    vals = []
    for b in range(len(theta)):
        S1, S2 = int(dims[b, 0]), int(dims[b, 1])
        A = orc.model_generator(1, theta[b], [S1, S2])
        rho = orc.expv_times(A, synth.delta(S1 * S2), T)
        lin = np.array([(j, x1 + S1 * x2, c) for j, x1, x2, c in recs])
        ll = orc.loglik(A, synth.delta(S1 * S2), T, lin)
        tol = sum(c * (2e-6 + 2e-9 / max(rho[j, s], 1e-300)) for j, s, c in lin)
        pmin = min(rho[j, s] for j, s, c in lin)
        vals.append((ll, tol, pmin))
    return vals


def check_vs_oracle(got, oracle_values, what):
    compared = 0
    for b, (ll, tol, pmin) in enumerate(oracle_values):
        if pmin < 1e-12:
            continue
        assert abs(got[b] - ll) <= tol, (what, b, got[b], ll, tol)
        compared += 1
    assert compared >= 12, compared


def test_every_shape_vs_oracle(mixed, oracle_values):
    theta, dims, T, recs = mixed
    shapes = mjp.mjp_loglik_shapes()
    lim = mjp.mjp_loglik_class_limits()
    assert [shape_class(int(a * b)) for a, b in GRIDS] == [0, 1, 2, 3]
    defaults = mjp.mjp_loglik_get_shapes(1, len(recs))
    for sid, sh in enumerate(shapes):
        ids = [sid if sh["max_states"] >= lim[c] else -1 for c in range(4)]
        mjp.mjp_loglik_set_shapes(1, ids)
        assert mjp.mjp_loglik_get_shapes(1, len(recs)) == [i if i >= 0 else d for i, d in zip(ids, defaults)]
        say(f"[gpu] loglik shape {sid} ({sh['threads']} x {sh['cells']}) on classes "
            f"{[c for c in range(4) if ids[c] >= 0]}")
        got = run(theta, dims, T, recs)
        check_vs_oracle(got, oracle_values, f"shape {sid}")


def test_tuner_report_and_choice(mixed, oracle_values):
    theta, dims, T, recs = mixed
    th = torch.as_tensor(np.asarray(theta, np.float64), device="cuda").contiguous()
    dm = torch.as_tensor(np.asarray(dims, np.int32), device="cuda").contiguous()
    out = torch.empty(len(theta), dtype=torch.float64, device="cuda")
    say("[gpu] loglik tune, 16 items over 4 classes")
    rep = mjp.mjp_loglik_tune(1, th, dm, mjp.make_obs(T, recs), out, reps=1)
    say(f"    items {rep['items']} chosen {rep['chosen']}")
    assert rep["items"] == [4, 4, 4, 4]
    shapes = mjp.mjp_loglik_shapes()
    lim = mjp.mjp_loglik_class_limits()
    for c in range(4):
        timed = {sid: rep["ms"][c][sid] for sid in range(len(shapes)) if rep["ms"][c][sid] >= 0}
        eligible = {sid for sid, sh in enumerate(shapes)
                    if sh["max_states"] >= lim[c] and len(recs) <= 4 * sh["threads"]}
        assert set(timed) == eligible, (c, timed, eligible)
        assert all(v > 0 for v in timed.values())
        assert rep["chosen"][c] == min(timed, key=timed.get)
        assert all(rep["ms"][c][sid] == -1.0 for sid in range(len(shapes), mjp.MJP_LL_MAX_SHAPES))
    assert mjp.mjp_loglik_get_shapes(1, len(recs)) == rep["chosen"]
    tuned = out.cpu().numpy()
    check_vs_oracle(tuned, oracle_values, "tuned")
    again = run(theta, dims, T, recs)              # mjp_loglik now uses the chosen shapes
    assert np.array_equal(tuned, again)


def test_record_capacity_falls_back_to_default():
    small = [10, 7, 4, -1]                          # 256-thread shapes: at most 1024 records
    assert all(mjp.mjp_loglik_shapes()[s]["threads"] == 256 for s in small[:3])
    mjp.mjp_loglik_set_shapes(1, small)
    assert mjp.mjp_loglik_get_shapes(1, 1024)[:3] == small[:3]
    default = mjp.mjp_loglik_get_shapes(1, 1025)
    mjp.mjp_loglik_set_shapes(1, [-1] * 4)
    assert default == mjp.mjp_loglik_get_shapes(1, 0)


def test_large_record_count_same_as_default(mixed):
    """1100 records (more than a 256-thread shape holds): the call with the
    small shapes set runs the defaults and gives their values bit for bit."""
    theta, dims, T, _ = mixed
    g = synth.rng(5)
    recs = np.stack([g.integers(0, 3, 1100), g.integers(0, 12, 1100), g.integers(0, 12, 1100),
                     np.ones(1100, np.int64)], axis=1)
    ref = run(theta, dims, T, recs)
    mjp.mjp_loglik_set_shapes(1, [10, 7, 4, -1])
    got = run(theta, dims, T, recs)
    assert np.array_equal(np.nan_to_num(ref, neginf=-1e300), np.nan_to_num(got, neginf=-1e300))


def test_unsorted_batch_groups_classes(mixed):
    """More items than the in-LDS sort takes (16,500): the order is grouped
    by class only; every item still gets the value it has in a small batch."""
    theta, dims, T, recs = mixed
    B = 16500
    g = synth.rng(9)
    th = np.asarray(theta)[g.integers(0, 16, B)]
    dm = np.tile(np.array([[20, 20]], np.int32), (B, 1))
    pick = [0, 4, 8, 12]                            # one item of each class at scattered slots
    slots = [3, 5000, 11000, 16499]
    for p, s in zip(pick, slots):
        th[s] = theta[p]
        dm[s] = dims[p]
    recs_small = recs[(recs[:, 1] < 20) & (recs[:, 2] < 20)]
    say(f"[gpu] loglik unsorted batch B={B}")
    big = run(th, dm, T, recs_small)
    sub = np.r_[slots, np.arange(100, 140)]
    ref = run(th[sub], dm[sub], T, recs_small)
    assert np.array_equal(np.nan_to_num(big[sub], neginf=-1e300), np.nan_to_num(ref, neginf=-1e300))


def test_shape_cache_round_trip(tmp_path):
    """The autotuner's on-disk cache: choices saved on this GPU load back
    exactly; a file keyed to another GPU is refused and changes nothing."""
    path = str(tmp_path / "shapes.txt")
    chosen = [10, 7, 4, -1]
    mjp.mjp_loglik_set_shapes(1, chosen)
    mjp.mjp_loglik_set_shapes(3, [-1, -1, 4, -1])
    want1, want3 = mjp.mjp_loglik_get_shapes(1), mjp.mjp_loglik_get_shapes(3)
    mjp.mjp_loglik_save_shapes(path)
    lines = open(path).read().splitlines()
    say("shape cache key:", lines[1])
    assert lines[0] == "mjp-loglik-shapes 1" and lines[1].startswith("gpu ") and len(lines) == 7
    assert lines[4] == "model 1 10 7 4 -1"
    mjp.mjp_loglik_set_shapes(1, [-1] * 4)
    mjp.mjp_loglik_set_shapes(3, [-1] * 4)
    mjp.mjp_loglik_load_shapes(path)
    assert mjp.mjp_loglik_get_shapes(1) == want1 and mjp.mjp_loglik_get_shapes(3) == want3
    other = list(lines)
    other[1] = "gpu gfx000 7 Another_GPU"
    other[4] = "model 1 -1 -1 -1 -1"
    p2 = str(tmp_path / "other.txt")
    open(p2, "w").write("\n".join(other) + "\n")
    with pytest.raises(mjp.MjpError) as e:
        mjp.mjp_loglik_load_shapes(p2)
    assert e.value.status == mjp.MJP_E_UNSUPPORTED
    assert mjp.mjp_loglik_get_shapes(1) == want1
    mjp.mjp_loglik_set_shapes(1, [-1] * 4)
    mjp.mjp_loglik_set_shapes(3, [-1] * 4)
