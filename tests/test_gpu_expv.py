"""GPU parity of mjp_expv against the FP64 oracle, through the C ABI.

Bar (FP32 products, FP64 weights): L1 distance <= 1e-6 per result vector, and
entrywise relative error <= 1e-4 wherever the oracle's probability exceeds
1e-7 (all terms are non-negative, so FP32 rounding stays relative; tiny
entries are dominated by the allowed left/right truncation of 2.5e-10 each).
"""
import math
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


def gpu_expv(plan, rho0, times, info=True):
    n = mjp.mjp_plan_n(plan)
    r0 = torch.as_tensor(np.asarray(rho0, np.float32), device="cuda")
    out = torch.empty((len(times), n), dtype=torch.float32, device="cuda")
    inf = mjp.mjp_expv(plan, r0, times, out, info=info)
    torch.cuda.synchronize()
    return out.cpu().double().numpy(), inf


def check_close(got, ref, what=""):
    l1 = np.abs(got - ref).sum()
    big = ref > 1e-7
    rel = (np.abs(got - ref)[big] / ref[big]).max() if big.any() else 0.0
    assert l1 <= L1_BAR, f"{what}: L1 {l1:.3e}"
    assert rel <= REL_BAR, f"{what}: entrywise rel {rel:.3e}"
    assert (got >= 0).all(), f"{what}: negative entry"
    return l1


def csr_plan_from_model(model, theta, dims, **opts):
    m = mjp.make_model(model, theta, dims)
    rp, ci, va = mjp.mjp_model_csr(m, opts.get("truncation", 0))
    return mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default(**opts))


def stencil_plan(model, theta, dims, **opts):
    return mjp.mjp_plan_create_stencil(mjp.make_model(model, theta, dims), mjp.mjp_opts_default(**opts))


@pytest.fixture(scope="module")
def bd_small(orc):
    """Immigration-death, N = 1000, lambda = 500, mu = 1, t = 1, from 0."""
    A = orc.model_generator(0, [500.0, 1.0], [1000])
    ref, info = orc.expv(A, synth.delta(1000), 1.0)
    return ref, info


VARIANTS = [mjp.MJP_VARIANT_STEPWISE, mjp.MJP_VARIANT_PERSISTENT, mjp.MJP_VARIANT_PERSISTENT_FENCED]
PERSISTENT = (mjp.MJP_VARIANT_PERSISTENT, mjp.MJP_VARIANT_PERSISTENT_FENCED)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("kind", ["csr", "stencil"])
def test_birth_death_small_workload(orc, bd_small, kind, variant):
    say(f"[gpu] birth-death N=1000 t=1 via {kind}, variant {variant}")
    ref, oinfo = bd_small
    plan = (csr_plan_from_model if kind == "csr" else stencil_plan)(0, [500.0, 1.0], [1000], variant=variant)
    try:
        got, inf = gpu_expv(plan, synth.delta(1000), [1.0])
    finally:
        mjp.mjp_plan_destroy(plan)
    check_close(got[0], ref, kind)
    from scipy.stats import poisson
    exact = poisson.pmf(np.arange(1000), 500.0 * (1 - math.exp(-1.0)))
    assert np.abs(got[0] - exact).sum() <= L1_BAR
    i = inf[0]
    assert abs(i["omega"] - oinfo["omega"]) < 1e-9 * oinfo["omega"]
    assert i["L"] > 0 and i["K"] > i["W"]
    assert i["eps_left"] <= 2.5e-10 and i["eps_right"] <= 2.5e-10
    assert abs(i["mass_in"] - 1) < 1e-7 and abs(i["mass_out"] - 1) < 1e-6 and i["flags"] == 0


@pytest.fixture(scope="module")
def cascade_300(orc):
    theta = [200.0, 1.0, 0.5, 0.5]
    A = orc.model_generator(1, theta, [300, 300])
    times = synth.log_spaced_times(16, 0.1, 10.0)
    say("[oracle] cascade 300x300, 16 times")
    ref = orc.expv_times(A, synth.delta(90000), times)
    return theta, times, ref


@pytest.mark.parametrize("variant", [mjp.MJP_VARIANT_AUTO, mjp.MJP_VARIANT_STEPWISE])
@pytest.mark.parametrize("kind", ["csr", "stencil"])
def test_cascade_16_times(cascade_300, kind, variant):
    theta, times, ref = cascade_300
    say(f"[gpu] cascade 300x300, 16 log-spaced times via {kind}, variant {variant}")
    plan = (csr_plan_from_model if kind == "csr" else stencil_plan)(1, theta, [300, 300], variant=variant)
    try:
        got, inf = gpu_expv(plan, synth.delta(90000), times)
    finally:
        mjp.mjp_plan_destroy(plan)
    worst = 0.0
    for j in range(len(times)):
        worst = max(worst, check_close(got[j], ref[j], f"{kind} t={times[j]:.3f}"))
        assert inf[j]["flags"] == 0
    say(f"    worst L1 over times: {worst:.3e}")


@pytest.mark.parametrize("variant", VARIANTS + [mjp.MJP_VARIANT_AUTO])
@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (63, 3), (64, 4), (65, 5), (257, 6), (1000, 7), (4097, 8),
                                    (33000, 10)])
def test_random_generators_ragged_sizes(orc, n, seed, variant):
    """Random sparse generators at sizes around the 64-row slice, the
    256-row block and the 512-row persistent workgroup: ragged tails."""
    say(f"[gpu] random generator n={n} seed={seed} variant {variant}")
    if n == 1:
        rp, ci, va = np.array([0, 1]), np.array([0]), np.array([0.0])
    else:
        rp, ci, va = synth.with_generator_diagonal(*synth.random_rate_graph(n, seed, degree=4, scale=3.0))
    A = orc.CSR.from_arrays(rp, ci, va)
    rho0 = synth.random_prob(n, seed + 50)
    times = [0.0, 0.05, 0.7, 2.3]
    ref = orc.expv_times(A, rho0, times)
    plan = mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default(variant=variant))
    pull_width = int(np.bincount(np.asarray(ci), minlength=n).max())  # incoming entries + diagonal
    try:
        if variant in PERSISTENT and pull_width > 16:
            # more incoming entries per state than the register budget holds
            with pytest.raises(mjp.MjpError) as e:
                gpu_expv(plan, rho0, times)
            assert e.value.status == mjp.MJP_E_UNSUPPORTED
            return
        got, inf = gpu_expv(plan, rho0, times)
    finally:
        mjp.mjp_plan_destroy(plan)
    for j, t in enumerate(times):
        check_close(got[j], ref[j], f"n={n} t={t}")
    assert np.array_equal(got[0], np.asarray(rho0, np.float32).astype(np.float64))  # t = 0 returns rho0


def test_unsorted_and_repeated_times(orc):
    A = orc.model_generator(1, [20.0, 1.0, 0.5, 0.5], [40, 30])
    rho0 = synth.delta(1200)
    times = [3.0, 0.5, 3.0, 0.0, 1e-9, 7.5]
    ref = orc.expv_times(A, rho0, times)
    say("[gpu] unsorted/repeated times")
    plan = stencil_plan(1, [20.0, 1.0, 0.5, 0.5], [40, 30])
    try:
        got, inf = gpu_expv(plan, rho0, times)
    finally:
        mjp.mjp_plan_destroy(plan)
    for j in range(len(times)):
        check_close(got[j], ref[j], f"t={times[j]}")
    assert np.array_equal(got[0], got[2])
    assert inf[4]["K"] <= 1


def test_zero_rates_return_rho0():
    say("[gpu] zero rates")
    plan = stencil_plan(1, [0.0, 0.0, 0.0, 0.0], [5, 4])
    rho0 = synth.random_prob(20, 3)
    try:
        got, inf = gpu_expv(plan, rho0, [0.0, 2.0])
    finally:
        mjp.mjp_plan_destroy(plan)
    r32 = np.asarray(rho0, np.float32).astype(np.float64)
    assert np.array_equal(got[0], r32) and np.array_equal(got[1], r32)
    assert inf[1]["omega"] == 0 and inf[1]["K"] == 0


@pytest.mark.parametrize("kind", ["csr", "stencil"])
def test_paper_rule_equal_K(orc, kind):
    """Paper cutoff K = floor(W + 6 sqrt W) + 1, accumulated from k = 0, on
    both sides: the GPU and the oracle run the same number of products."""
    say(f"[gpu] paper cutoff via {kind}")
    A = orc.model_generator(0, [60.0, 2.0], [150])
    rho0 = synth.delta(150, 3)
    ref, oi = orc.expv(A, rho0, 0.3, k_rule=orc.K_PAPER)
    mk = csr_plan_from_model if kind == "csr" else stencil_plan
    plan = mk(0, [60.0, 2.0], [150], k_rule=mjp.MJP_K_PAPER)
    try:
        got, inf = gpu_expv(plan, rho0, [0.3])
    finally:
        mjp.mjp_plan_destroy(plan)
    assert inf[0]["K"] == oi["K"] and inf[0]["L"] == 0
    check_close(got[0], ref, "paper rule")


def test_without_lumping_mass_is_window_weight(orc):
    say("[gpu] lump off")
    plan = stencil_plan(1, [30.0, 1.0, 0.5, 0.5], [60, 50], lump=0, tol=1e-4)
    try:
        got, inf = gpu_expv(plan, synth.delta(3000), [1.5])
    finally:
        mjp.mjp_plan_destroy(plan)
    i = inf[0]
    assert i["residual"] > 1e-6
    assert abs(got[0].sum() - (1 - i["residual"])) < 2e-7
    assert abs(i["mass_out"] - (1 - i["residual"])) < 2e-7


@pytest.mark.parametrize("factor", [1.5, 2.0])
def test_omega_factor(orc, factor):
    say(f"[gpu] omega factor {factor}")
    A = orc.model_generator(1, [15.0, 1.0, 0.6, 0.4], [35, 40])
    rho0 = synth.random_prob(1400, 9)
    ref, _ = orc.expv(A, rho0, 1.2, omega_factor=factor)
    plan = stencil_plan(1, [15.0, 1.0, 0.6, 0.4], [35, 40], omega_factor=factor)
    try:
        got, inf = gpu_expv(plan, rho0, [1.2])
    finally:
        mjp.mjp_plan_destroy(plan)
    check_close(got[0], ref, f"factor {factor}")


@pytest.mark.parametrize("renorm", [0, 1, 7])
def test_renorm_interval(orc, renorm):
    say(f"[gpu] renorm_every={renorm}")
    A = orc.model_generator(1, [40.0, 1.0, 0.5, 0.5], [80, 70])
    rho0 = synth.delta(5600)
    ref, _ = orc.expv(A, rho0, 4.0)
    plan = stencil_plan(1, [40.0, 1.0, 0.5, 0.5], [80, 70], renorm_every=renorm)
    try:
        got, _ = gpu_expv(plan, rho0, [4.0])
    finally:
        mjp.mjp_plan_destroy(plan)
    check_close(got[0], ref, f"renorm {renorm}")


def test_leaky_truncation(orc):
    """Leaky reading (exit rate counts births off the grid): mass leaks; the
    oracle's leaky generator is the reference."""
    say("[gpu] leaky truncation")
    A = orc.model_generator(0, [30.0, 1.0], [40], leaky=True)
    ref, _ = orc.expv(A, synth.delta(40), 2.0)
    for kind in ("csr", "stencil"):
        mk = csr_plan_from_model if kind == "csr" else stencil_plan
        plan = mk(0, [30.0, 1.0], [40], truncation=mjp.MJP_LEAKY, renorm_every=0)
        try:
            got, _ = gpu_expv(plan, synth.delta(40), [2.0])
        finally:
            mjp.mjp_plan_destroy(plan)
        assert ref.sum() < 0.999
        check_close(got[0], ref, f"leaky {kind}")


@pytest.mark.parametrize("variant", VARIANTS)
def test_bitwise_deterministic(variant):
    say(f"[gpu] determinism, variant {variant}")
    plan = csr_plan_from_model(1, [200.0, 1.0, 0.5, 0.5], [120, 150], variant=variant)
    try:
        a, _ = gpu_expv(plan, synth.delta(18000), [0.3, 2.0], info=False)
        b, _ = gpu_expv(plan, synth.delta(18000), [0.3, 2.0], info=False)
    finally:
        mjp.mjp_plan_destroy(plan)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("bad,flag", [(np.nan, mjp.MJP_FLAG_NAN), (-0.25, mjp.MJP_FLAG_NEG)])
def test_bad_rho0_flags(bad, flag):
    say(f"[gpu] rho0 with {bad}")
    plan = stencil_plan(0, [5.0, 1.0], [30])
    rho0 = synth.random_prob(30, 4)
    rho0[7] = bad
    r0 = torch.as_tensor(rho0.astype(np.float32), device="cuda")
    out = torch.empty((1, 30), dtype=torch.float32, device="cuda")
    try:
        with pytest.raises(mjp.MjpError) as e:
            mjp.mjp_expv(plan, r0, [1.0], out, info=True)
        assert e.value.status == mjp.MJP_E_NUMERIC
        # asynchronous form does not fail, it only computes
        mjp.mjp_expv(plan, r0, [1.0], out, info=False)
        torch.cuda.synchronize()
    finally:
        mjp.mjp_plan_destroy(plan)


def test_k_cap():
    plan = stencil_plan(0, [500.0, 1.0], [1000], k_cap=100)
    r0 = torch.zeros(1000, device="cuda")
    out = torch.empty((1, 1000), device="cuda")
    try:
        with pytest.raises(mjp.MjpError) as e:
            mjp.mjp_expv(plan, r0, [1.0], out)
        assert e.value.status == mjp.MJP_E_K_LIMIT
    finally:
        mjp.mjp_plan_destroy(plan)


def test_batched_matches_single(orc):
    say("[gpu] expv_batched")
    plans = [stencil_plan(0, [50.0, 1.0], [200]), stencil_plan(1, [10.0, 1.0, 0.5, 0.5], [30, 30]),
             csr_plan_from_model(1, [5.0, 1.0, 2.0, 1.0], [20, 41])]
    rho0s = [synth.delta(200), synth.random_prob(900, 1), synth.random_prob(820, 2)]
    times = [[0.5, 2.0], [1.0], [0.2, 0.9, 3.0]]
    try:
        r = [torch.as_tensor(x.astype(np.float32), device="cuda") for x in rho0s]
        outs = [torch.empty((len(t), mjp.mjp_plan_n(p)), device="cuda") for p, t in zip(plans, times)]
        inf = mjp.mjp_expv_batched(plans, r, times, outs, info=True)
        torch.cuda.synchronize()
        assert len(inf) == 6
        refs = [orc.expv_times(orc.model_generator(0, [50.0, 1.0], [200]), rho0s[0], times[0]),
                orc.expv_times(orc.model_generator(1, [10.0, 1.0, 0.5, 0.5], [30, 30]), rho0s[1], times[1]),
                orc.expv_times(orc.model_generator(1, [5.0, 1.0, 2.0, 1.0], [20, 41]), rho0s[2], times[2])]
        for o, ref in zip(outs, refs):
            o = o.cpu().double().numpy()
            for j in range(len(ref)):
                check_close(o[j], ref[j], "batched")
    finally:
        for p in plans:
            mjp.mjp_plan_destroy(p)


def test_persistent_refuses_wide_operator():
    """A generator with rows wider than the register budget is refused by the
    persistent variant (and solved by the stepwise one under AUTO)."""
    rp, ci, va = synth.with_generator_diagonal(*synth.random_rate_graph(24, 5, dense=True, scale=1.0))
    plan = mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default(variant=mjp.MJP_VARIANT_PERSISTENT))
    r0 = torch.full((24,), 1.0 / 24, device="cuda")
    out = torch.empty((1, 24), device="cuda")
    try:
        with pytest.raises(mjp.MjpError) as e:
            mjp.mjp_expv(plan, r0, [0.5], out)
        assert e.value.status == mjp.MJP_E_UNSUPPORTED
    finally:
        mjp.mjp_plan_destroy(plan)


def _protocol_case(name):
    """(plan factory, rho0, times) for the protocol comparison."""
    if name == "cascade-csr-90000":
        return (lambda **o: csr_plan_from_model(1, [60.0, 1.0, 0.7, 0.4], [300, 300], **o),
                synth.delta(90000), [0.05, 2.0, 2.1, 2.2, 2.3])  # up to 4 windows open together
    if name == "cascade-stencil-90000":
        return (lambda **o: stencil_plan(1, [60.0, 1.0, 0.7, 0.4], [300, 300], **o),
                synth.random_prob(90000, 3), [0.4, 2.5])
    if name == "bd-stencil-1000":
        return (lambda **o: stencil_plan(0, [500.0, 1.0], [1000], **o), synth.delta(1000), [1.0])
    if name == "random-csr-33000":
        rp, ci, va = synth.with_generator_diagonal(*synth.random_rate_graph(33000, 10, degree=4, scale=3.0))
        return (lambda **o: mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default(**o)),
                synth.random_prob(33000, 60), [0.05, 0.7, 2.3])
    if name == "banded-csr-200001":
        # a ragged size (not a multiple of the 4096-row workgroup) with narrow
        # neighbour intervals: the flags path, not the global barrier
        m = mjp.make_model(1, [30.0, 1.0, 1.0, 0.5], [401, 499])
        rp, ci, va = mjp.mjp_model_csr(m)
        return (lambda **o: mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default(**o)),
                synth.random_prob(401 * 499, 61), [0.3, 1.1])
    raise KeyError(name)


@pytest.mark.parametrize("renorm", [32, 0, 1])
@pytest.mark.parametrize("case", ["cascade-csr-90000", "cascade-stencil-90000", "bd-stencil-1000",
                                  "random-csr-33000", "banded-csr-200001"])
def test_protocols_bit_identical(case, renorm):
    """The persistent kernel's two memory protocols (device-scope iterate
    accesses vs agent-scope fences) do the same arithmetic in the same order,
    so their results must agree bit for bit; a stale read of the iterate in
    either would change the bits.  renorm 0 runs on neighbour flags only,
    renorm 1 on a grid barrier every jump."""
    make, rho0, times = _protocol_case(case)
    say(f"[gpu] protocols {case} renorm_every={renorm}")
    res = []
    for variant in PERSISTENT:
        plan = make(variant=variant, renorm_every=renorm)
        try:
            res.append(gpu_expv(plan, rho0, times, info=False)[0])
        finally:
            mjp.mjp_plan_destroy(plan)
    assert np.array_equal(res[0], res[1])


def _twojump_case(name):
    """(plan factory, rho0, times, whether the two-jump kernel can hold it)."""
    cas = mjp.make_model(1, [30.0, 1.0, 1.0, 0.5], [700, 800])
    rp, ci, va = mjp.mjp_model_csr(cas)
    if name == "cascade-csr-560000":          # two windows open together
        return (lambda **o: mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default(**o)),
                synth.delta(560000), [0.05, 0.3, 0.31], True)
    if name == "cascade-csr-560000-3open":    # three: more than the two-jump kernel keeps
        return (lambda **o: mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default(**o)),
                synth.delta(560000), [0.3, 0.31, 0.32], False)
    if name == "cascade-stencil-600000-odd":
        m = mjp.make_model(1, [30.0, 1.0, 0.7, 0.4], [600, 1000])
        return (lambda **o: mjp.mjp_plan_create_stencil(m, mjp.mjp_opts_default(**o)),
                synth.random_prob(600000, 71), [0.2], True)
    if name == "bd-stencil-700001":
        m = mjp.make_model(0, [50000.0, 0.01], [700001])
        return (lambda **o: mjp.mjp_plan_create_stencil(m, mjp.mjp_opts_default(**o)),
                synth.delta(700001), [0.01, 0.013], True)
    raise KeyError(name)


@pytest.mark.parametrize("renorm", [32, 0, 2, 1])
@pytest.mark.parametrize("case", ["cascade-csr-560000", "cascade-csr-560000-3open", "cascade-stencil-600000-odd",
                                  "bd-stencil-700001"])
def test_twojump_bit_identical(case, renorm):
    """Two jumps per synchronisation (neighbours' boundary rows recomputed
    from the same inputs with the same operations) against the one-jump
    kernel and the fenced protocol, bit for bit, on operators large enough
    for the two-jump kernel (>= 128 workgroups of 4096 rows; ragged sizes;
    odd and even jump counts; two windows open together).  An odd
    renorm_every cannot end a two-jump round, and more than two open windows
    exceed its registers: those sweeps fall back to one jump per
    synchronisation."""
    make, rho0, times, fits = _twojump_case(case)
    say(f"[gpu] two-jump {case} renorm_every={renorm}")
    res, paths = [], []
    for variant in (mjp.MJP_VARIANT_PERSISTENT_TWOJUMP, mjp.MJP_VARIANT_PERSISTENT_ONEJUMP,
                    mjp.MJP_VARIANT_PERSISTENT_FENCED):
        plan = make(variant=variant, renorm_every=renorm)
        try:
            out, inf = gpu_expv(plan, rho0, times, info=True)
        finally:
            mjp.mjp_plan_destroy(plan)
        res.append(out)
        paths.append(inf[0]["path"])
        say(f"    variant {variant}: path {inf[0]['path']}, K {[i['K'] for i in inf]}")
    want = mjp.MJP_PATH_PERSISTENT_TWOJUMP if fits and renorm % 2 == 0 else mjp.MJP_PATH_PERSISTENT
    assert paths == [want, mjp.MJP_PATH_PERSISTENT, mjp.MJP_PATH_PERSISTENT_FENCED]
    for r in res[1:]:
        assert np.array_equal(res[0], r)


@pytest.mark.parametrize("dims", [(1000, 1000), (750, 750)])
def test_wait_deadline_abort_path(dims):
    """The abort path of the two-jump kernel, forced from the host: with
    barrier_timeout_us < 0 it runs in a form whose grid and neighbour waits
    give up at their first unready read, raising the abort flag, so every
    workgroup leaves the kernel; the call with info reports MJP_E_DEVICE.
    A solve with the default deadline afterwards is bit-identical to one
    before (nothing is left behind)."""
    variant = mjp.MJP_VARIANT_PERSISTENT_TWOJUMP
    S1, S2 = dims
    n = S1 * S2
    rp, ci, va = mjp.mjp_model_csr(mjp.make_model(mjp.MJP_MODEL_CASCADE2, [200.0, 1.0, 0.5, 0.5], [S1, S2]))
    rho0 = np.zeros(n, np.float32)
    rho0[0] = 1.0

    def solve(**opts):
        plan = mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default(variant=variant, **opts))
        try:
            return gpu_expv(plan, rho0, [1.0], info=True)
        finally:
            mjp.mjp_plan_destroy(plan)

    say(f"[gpu] wait-deadline abort path: variant {variant}, {S1}x{S2}")
    before, inf = solve()
    assert inf[0]["path"] == mjp.MJP_PATH_PERSISTENT_TWOJUMP
    with pytest.raises(mjp.MjpError) as e:
        solve(barrier_timeout_us=-1)
    assert e.value.status == mjp.MJP_E_DEVICE and "timed out" in str(e.value)
    after, _ = solve()
    assert np.array_equal(before, after)


@pytest.mark.parametrize("kind", ["csr", "stencil"])
def test_tiled_sweep_mid_size(orc, kind):
    """A 300 x 300 cascade (N = 90,000, 22 tiles of the grid) at one time
    runs the tiled sweep (eight jumps per neighbour exchange): it meets the
    parity bar against the FP64 oracle and equals the one-jump kernel bit
    for bit."""
    theta = [200.0, 1.0, 0.5, 0.5]
    A = orc.model_generator(1, theta, [300, 300])
    say(f"[oracle] cascade 300x300, t=10")
    ref, _ = orc.expv(A, synth.delta(90000), 10.0)
    outs, paths = [], []
    for variant in (mjp.MJP_VARIANT_AUTO, mjp.MJP_VARIANT_PERSISTENT_ONEJUMP):
        say(f"[gpu] cascade 300x300 t=10 via {kind}, variant {variant}")
        plan = (csr_plan_from_model if kind == "csr" else stencil_plan)(1, theta, [300, 300], variant=variant)
        try:
            got, inf = gpu_expv(plan, synth.delta(90000), [10.0])
        finally:
            mjp.mjp_plan_destroy(plan)
        outs.append(got)
        paths.append(inf[0]["path"])
        assert inf[0]["flags"] == 0
    assert paths == [mjp.MJP_PATH_PERSISTENT_MULTIJUMP, mjp.MJP_PATH_PERSISTENT]
    say(f"    L1 {check_close(outs[0][0], ref, kind):.3e}")
    assert np.array_equal(outs[0], outs[1])
