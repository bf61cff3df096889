"""mjp_expv_batched through the C ABI: the batched item sweep (one workgroup
per item, one launch per operator class) against each item's own mjp_expv
call (bit for bit) and against the FP64 oracle (the bar of
test_gpu_expv.py: L1 <= 1e-6, entrywise relative <= 1e-4 above 1e-7).

Items: the immigration-death process at N = 1000 (lambda 500, mu 1, the
single-vector workload), the cascade on small grids (stencil and CSR plans),
the two-state and autoregulatory gene models, random sparse generators
(ragged sizes), plus items the batched sweep cannot hold (too many rows,
too many times, the stepwise variant), which run their own sweep.
"""
import sys

import numpy as np
import pytest
import torch

from paper_2312_05647_amd import mjp, synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

L1_BAR = 1e-6
REL_BAR = 1e-4


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def check_close(got, ref, what=""):
    l1 = np.abs(got - ref).sum()
    big = ref > 1e-7
    rel = (np.abs(got - ref)[big] / ref[big]).max() if big.any() else 0.0
    assert l1 <= L1_BAR, f"{what}: L1 {l1:.3e}"
    assert rel <= REL_BAR, f"{what}: entrywise rel {rel:.3e}"
    assert (got >= 0).all(), f"{what}: negative entry"


def stencil_plan(model, theta, dims, **opts):
    return mjp.mjp_plan_create_stencil(mjp.make_model(model, theta, dims), mjp.mjp_opts_default(**opts))


def csr_plan_from_model(model, theta, dims, **opts):
    rp, ci, va = mjp.mjp_model_csr(mjp.make_model(model, theta, dims), 0)
    return mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default(**opts))


def csr_plan_random(n, seed, **opts):
    if n == 1:
        rp, ci, va = np.array([0, 1]), np.array([0], np.int32), np.array([0.0])
    else:
        rp, ci, va = synth.with_generator_diagonal(*synth.random_rate_graph(n, seed))
    return mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default(**opts)), (rp, ci, va)


def held_by_one_workgroup(n, ci):
    """The batched sweep's rule for a CSR plan: entries per pulled row
    (incoming rates + the diagonal) padded to 3, 5, 8, 12 or 16, and up to
    512 R rows with R <= 8, 8, 4, 4, 2 for those widths."""
    width = int(np.bincount(np.asarray(ci), minlength=n).max())
    for W, R in ((3, 8), (5, 8), (8, 4), (12, 4), (16, 2)):
        if width <= W:
            return n <= 512 * R
    return False


def run_batched(plans, rho0s, times, info=True):
    r = [torch.as_tensor(np.asarray(x, np.float32), device="cuda") for x in rho0s]
    outs = [torch.full((len(t), mjp.mjp_plan_n(p)), -1.0, device="cuda") for p, t in zip(plans, times)]
    inf = mjp.mjp_expv_batched(plans, r, times, outs, info=info)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs], inf


def run_single(plan, rho0, times):
    r = torch.as_tensor(np.asarray(rho0, np.float32), device="cuda")
    out = torch.full((len(times), mjp.mjp_plan_n(plan)), -1.0, device="cuda")
    inf = mjp.mjp_expv(plan, r, times, out, info=True)
    torch.cuda.synchronize()
    return out.cpu().numpy(), inf


@pytest.fixture(scope="module")
def mixed(orc):
    """Items of every kind the batched sweep holds, plus three it does not."""
    items = []  # (plan, rho0, times, oracle generator or None, expect batched)
    items.append((stencil_plan(0, [500.0, 1.0], [1000]), synth.delta(1000), [1.0],
                  orc.model_generator(0, [500.0, 1.0], [1000]), True))
    items.append((stencil_plan(1, [10.0, 1.0, 0.5, 0.5], [30, 30]), synth.random_prob(900, 1), [0.3, 1.0, 4.0],
                  orc.model_generator(1, [10.0, 1.0, 0.5, 0.5], [30, 30]), True))
    items.append((csr_plan_from_model(1, [5.0, 1.0, 2.0, 1.0], [20, 41]), synth.random_prob(820, 2), [0.2, 0.9, 3.0],
                  orc.model_generator(1, [5.0, 1.0, 2.0, 1.0], [20, 41]), True))
    items.append((stencil_plan(2, [20.0, 1.0, 0.7, 0.3], [120]), synth.delta(240), [0.5, 2.0, 10.0],
                  orc.model_generator(2, [20.0, 1.0, 0.7, 0.3], [120]), True))
    th_ar = [10.0, 5.0, 1.0, 1.0, 0.3, 0.02]
    items.append((stencil_plan(3, th_ar, [24, 40]), synth.delta(2 * 24 * 40), [0.5, 3.0],
                  orc.model_generator(3, th_ar, [24, 40]), True))
    for n, seed in [(1, 11), (63, 12), (65, 13), (513, 14), (2048, 15), (4096, 17)]:
        p, (rp, ci, va) = csr_plan_random(n, seed)
        items.append((p, synth.random_prob(n, seed), [0.05, 0.4], orc.CSR.from_arrays(rp, ci, va),
                      held_by_one_workgroup(n, ci)))
    # not held by one workgroup: more rows, more than 48 times, the stepwise variant
    p, (rp, ci, va) = csr_plan_random(4097, 16)
    items.append((p, synth.random_prob(4097, 16), [0.3], orc.CSR.from_arrays(rp, ci, va), False))
    items.append((stencil_plan(0, [50.0, 1.0], [200]), synth.delta(200), list(np.linspace(0.05, 3.0, 50)),
                  orc.model_generator(0, [50.0, 1.0], [200]), False))
    items.append((stencil_plan(0, [50.0, 1.0], [200], variant=mjp.MJP_VARIANT_STEPWISE), synth.delta(200), [1.0],
                  orc.model_generator(0, [50.0, 1.0], [200]), False))
    yield items
    for it in items:
        mjp.mjp_plan_destroy(it[0])


def test_mixed_batch_equals_single_calls_and_oracle(orc, mixed):
    say("[gpu] expv_batched: mixed batch")
    plans = [it[0] for it in mixed]
    rho0s = [it[1] for it in mixed]
    times = [it[2] for it in mixed]
    outs, inf = run_batched(plans, rho0s, times)
    assert len(inf) == sum(len(t) for t in times)
    off = 0
    for b, (plan, rho0, ts, A, batched) in enumerate(mixed):
        ref_gpu, ref_inf = run_single(plan, rho0, ts)
        for j in range(len(ts)):
            e = inf[off + j]
            assert (e["path"] == mjp.MJP_PATH_BATCHED_ITEM) == batched, (b, e["path"])
            assert e["K"] == ref_inf[j]["K"] and e["L"] == ref_inf[j]["L"]
            assert abs(e["mass_out"] - outs[b][j].astype(np.float64).sum()) <= 1e-6
        if batched:
            # the batched sweep is the single-workgroup sweep: same bits
            assert np.array_equal(outs[b].view(np.uint32), ref_gpu.view(np.uint32)), f"item {b} differs from mjp_expv"
        ref = orc.expv_times(A, np.asarray(rho0, np.float64), ts)
        for j in range(len(ts)):
            check_close(outs[b][j].astype(np.float64), ref[j], f"item {b} time {ts[j]}")
        off += len(ts)


def test_many_items_through_the_queue(orc):
    """More items than resident workgroups, one plan repeated with different
    initial vectors, two calls in a row on one stream (the second smaller and
    without info), and an asynchronous call before a synchronous one."""
    say("[gpu] expv_batched: queue")
    plan = stencil_plan(0, [40.0, 1.0], [128])
    A = orc.model_generator(0, [40.0, 1.0], [128])
    try:
        g = synth.rng(5)
        B = 3000
        rho0s = [g.dirichlet(np.ones(128)) for _ in range(B)]
        times = [[float(t)] for t in g.uniform(0.1, 2.0, B)]
        outs, inf = run_batched([plan] * B, rho0s, times)
        assert all(e["path"] == mjp.MJP_PATH_BATCHED_ITEM for e in inf)
        for b in list(range(0, B, 397)) + [B - 1]:
            ref = orc.expv_times(A, rho0s[b], times[b])
            check_close(outs[b][0].astype(np.float64), ref[0], f"item {b}")
            single, _ = run_single(plan, rho0s[b], times[b])
            assert np.array_equal(outs[b].view(np.uint32), single.view(np.uint32))
        # second call: fewer items, no info (asynchronous), then read
        outs2, _ = run_batched([plan] * 7, rho0s[:7], times[:7], info=False)
        for b in range(7):
            assert np.array_equal(outs2[b].view(np.uint32), outs[b].view(np.uint32))
    finally:
        mjp.mjp_plan_destroy(plan)


def test_bad_item_reports_numeric_flag():
    say("[gpu] expv_batched: NaN item")
    plan = stencil_plan(0, [40.0, 1.0], [128])
    try:
        good = synth.delta(128)
        bad = synth.delta(128)
        bad[3] = np.nan
        with pytest.raises(mjp.MjpError) as e:
            run_batched([plan, plan], [good, bad], [[1.0], [1.0]])
        assert e.value.status == mjp.MJP_E_NUMERIC
        # the library stays usable
        outs, inf = run_batched([plan], [good], [[1.0]])
        assert inf[0]["flags"] == 0 and abs(outs[0][0].sum() - 1.0) < 1e-5
    finally:
        mjp.mjp_plan_destroy(plan)
