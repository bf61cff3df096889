"""The allocation-free log-likelihood call (mjp_loglik_noalloc: the call's
tables in the library's fixed per-GPU device array) through the C ABI: two
calls in a row, the second with fewer items, other times and other
records, each equal bit for bit to mjp_loglik on the same inputs (same
kernels and launch shapes; its arguments differ only in where the tables
live)."""
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


def case(n_draws, n_times, snaps, seed, theta_star):
    T = synth.even_times(n_times, 0.5)
    data = synth.gillespie_cascade2(theta_star, T, snaps, seed=seed)
    recs = synth.cascade_records(data)
    theta = synth.theta_draws(n_draws, theta_star, seed=seed + 1)
    dims = synth.grid_dims(theta, (int(data[:, 1].max()), int(data[:, 2].max())), lo=20, hi=60)
    return theta, dims, T, recs


def both(theta, dims, T, recs):
    B = len(theta)
    th = torch.as_tensor(theta, device="cuda")
    dm = torch.as_tensor(np.asarray(dims, np.int32), device="cuda")
    obs = mjp.make_obs(T, recs, (0, 0))
    sz = ctypes.sizeof(mjp.mjp_info)
    res = []
    for fn in (mjp.mjp_loglik, mjp.mjp_loglik_noalloc):
        out = torch.full((B,), 7.0, dtype=torch.float64, device="cuda")
        info = torch.zeros(B * sz, dtype=torch.uint8, device="cuda")
        fn(1, th, dm, obs, out, info=info)
        torch.cuda.synchronize()
        res.append((out.cpu().numpy(), info.cpu().numpy()))
    return res


def test_noalloc_equals_allocating_call_twice():
    cap = mjp.mjp_loglik_noalloc_capacity()
    big = case(600, 12, 20, 1001, [16.0, 1.0, 0.6, 0.5])
    small = case(70, 5, 9, 2002, [10.0, 0.7, 0.5, 0.6])
    for name, (theta, dims, T, recs) in (("first", big), ("second, smaller", small)):
        need = mjp.mjp_loglik_noalloc_bytes(len(theta), len(T), len(recs))
        say(f"[gpu] noalloc {name}: B={len(theta)}, {len(T)} times, {len(recs)} records, {need} of {cap} bytes")
        assert 0 < need <= cap
        (a, ia), (b, ib) = both(theta, dims, T, recs)
        assert np.isfinite(a).mean() > 0.5
        assert np.array_equal(a, b), (name, np.flatnonzero(a != b)[:5])
        assert np.array_equal(ia, ib), name
