"""Full-size parity: two-species cascade on a 1000 x 1000 grid (N = 10^6,
4,995,001 stored entries), rates (200, 1, 0.5, 0.5), rho(0) at (0, 0), t = 1,
in the configuration the benchmark times.  Compared element by element with
the FP64 oracle (a full solve, ~10 s on the host), and with the closed-form
species-1 marginal Poisson(200 (1 - e^{-1}))."""
import math
import sys

import numpy as np
import pytest
import torch
from scipy.stats import poisson

from paper_2312_05647_amd import mjp, synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

THETA = [200.0, 1.0, 0.5, 0.5]
S = 1000


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ref(orc):
    say(f"[oracle] cascade {S}x{S} t=1 on {orc.num_threads()} threads")
    A = orc.model_generator(1, THETA, [S, S])
    out, info = orc.expv(A, synth.delta(S * S), 1.0)
    return out, info


def run(plan):
    r0 = torch.zeros(S * S, device="cuda")
    r0[0] = 1.0
    out = torch.empty((1, S * S), device="cuda")
    inf = mjp.mjp_expv(plan, r0, [1.0], out, info=True)
    torch.cuda.synchronize()
    return out[0].cpu().double().numpy(), inf[0]


@pytest.mark.parametrize("kind", ["csr", "stencil"])
@pytest.mark.parametrize("variant", [mjp.MJP_VARIANT_PERSISTENT, mjp.MJP_VARIANT_PERSISTENT_TWOJUMP,
                                     mjp.MJP_VARIANT_PERSISTENT_FENCED, mjp.MJP_VARIANT_PERSISTENT_ONEJUMP,
                                     mjp.MJP_VARIANT_STEPWISE])
def test_full_size_parity(ref, kind, variant):
    say(f"[gpu] cascade {S}x{S} t=1 via {kind}, variant {variant}")
    m = mjp.make_model(1, THETA, [S, S])
    opts = mjp.mjp_opts_default(variant=variant)
    if kind == "csr":
        plan = mjp.mjp_plan_create_csr(*mjp.mjp_model_csr(m), opts)
    else:
        plan = mjp.mjp_plan_create_stencil(m, opts)
    try:
        got, inf = run(plan)
    finally:
        mjp.mjp_plan_destroy(plan)
    oref, oinfo = ref
    l1 = np.abs(got - oref).sum()
    big = oref > 1e-7
    rel = (np.abs(got - oref)[big] / oref[big]).max()
    say(f"    L1 {l1:.3e}  Linf {np.abs(got - oref).max():.3e}  rel(p>1e-7) {rel:.3e}  K {inf['K']} L {inf['L']}")
    assert l1 <= 1e-6
    assert rel <= 1e-4
    assert (got >= 0).all()
    assert abs(inf["omega"] - oinfo["omega"]) < 1e-9 * oinfo["omega"]
    assert abs(inf["mass_out"] - 1.0) < 1e-6 and inf["flags"] == 0
    # species-1 marginal against the immigration-death closed form
    marg = got.reshape(S, S).sum(axis=0)
    exact = poisson.pmf(np.arange(S), THETA[0] * (1 - math.exp(-1.0)))
    assert np.abs(marg - exact).sum() <= 1e-6


@pytest.mark.parametrize("kind", ["csr", "stencil"])
def test_full_size_protocols_bit_identical(kind):
    """The persistent kernel's forms (eight jumps per synchronisation on
    tiles, two on row blocks, one jump with device-scope accesses, one jump
    with fences) agree bit for bit at full size (every XCD)."""
    say(f"[gpu] cascade {S}x{S} protocols via {kind}")
    m = mjp.make_model(1, THETA, [S, S])
    res, paths = [], []
    for variant in (mjp.MJP_VARIANT_PERSISTENT, mjp.MJP_VARIANT_PERSISTENT_TWOJUMP,
                    mjp.MJP_VARIANT_PERSISTENT_FENCED, mjp.MJP_VARIANT_PERSISTENT_ONEJUMP):
        opts = mjp.mjp_opts_default(variant=variant)
        plan = mjp.mjp_plan_create_csr(*mjp.mjp_model_csr(m), opts) if kind == "csr" else \
            mjp.mjp_plan_create_stencil(m, opts)
        try:
            out, inf = run(plan)
            res.append(out)
            paths.append(inf["path"])
        finally:
            mjp.mjp_plan_destroy(plan)
    assert paths == [mjp.MJP_PATH_PERSISTENT_MULTIJUMP, mjp.MJP_PATH_PERSISTENT_TWOJUMP,
                     mjp.MJP_PATH_PERSISTENT_FENCED, mjp.MJP_PATH_PERSISTENT]
    for r in res[1:]:
        assert np.array_equal(res[0], r)


def _mj_case(name):
    """(plan factory, rho0, times) of grids large enough for the tiled kernel."""
    if name == "cascade-csr-1000x1000-2open":
        m = mjp.make_model(1, THETA, [S, S])
        rp, ci, va = mjp.mjp_model_csr(m)
        return (lambda **o: mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default(**o)),
                synth.delta(S * S), [0.3, 0.31])
    if name == "cascade-stencil-750x750-random":
        m = mjp.make_model(1, [30.0, 1.0, 0.7, 0.4], [750, 750])
        return (lambda **o: mjp.mjp_plan_create_stencil(m, mjp.mjp_opts_default(**o)),
                synth.random_prob(750 * 750, 72), [0.21])
    if name == "cascade-csr-600x1500":
        m = mjp.make_model(1, [40.0, 1.0, 0.6, 0.5], [600, 1500])
        rp, ci, va = mjp.mjp_model_csr(m)
        return (lambda **o: mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default(**o)),
                synth.random_prob(600 * 1500, 73), [0.05, 0.4])
    if name == "birth-csr-1000x1000":
        # death rates 0: the builder drops the zero entries, so every row reads
        # only the states below it and a tile's reads across a side go one way
        m = mjp.make_model(1, [30.0, 0.0, 0.7, 0.0], [S, S])
        rp, ci, va = mjp.mjp_model_csr(m)
        return (lambda **o: mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default(**o)),
                synth.random_prob(S * S, 74), [0.2, 0.35])
    if name == "bd-stencil-700001":
        m = mjp.make_model(0, [50000.0, 0.01], [700001])
        return (lambda **o: mjp.mjp_plan_create_stencil(m, mjp.mjp_opts_default(**o)),
                synth.delta(700001), [0.01, 0.013])
    raise KeyError(name)


@pytest.mark.parametrize("renorm", [32, 0, 4, 8, 2])
@pytest.mark.parametrize("case", ["cascade-csr-1000x1000-2open", "cascade-stencil-750x750-random",
                                  "cascade-csr-600x1500", "bd-stencil-700001", "birth-csr-1000x1000"])
def test_multijump_bit_identical(case, renorm):
    """Four jumps per synchronisation on tiles (rings of cells around each
    tile recomputed from the same inputs with the same operations) against
    the one-jump kernel, bit for bit: square and oblong grids, CSR and
    stencil plans, a band operator (1-D blocks), an operator whose rows
    read only lower states (a tile waits for the tiles it reads and for those
    that read it), jump counts of every residue mod 4, two windows open
    together, renormalisation every 4, 8 or 32 jumps or never.  renorm_every = 2 cannot end a four-jump round: the
    sweep then takes the two-jump kernel."""
    make, rho0, times = _mj_case(case)
    say(f"[gpu] multi-jump {case} renorm_every={renorm}")
    res, paths = [], []
    for variant in (mjp.MJP_VARIANT_PERSISTENT, mjp.MJP_VARIANT_PERSISTENT_ONEJUMP):
        plan = make(variant=variant, renorm_every=renorm)
        try:
            r0 = torch.as_tensor(np.asarray(rho0, np.float32), device="cuda")
            out = torch.empty((len(times), mjp.mjp_plan_n(plan)), device="cuda")
            inf = mjp.mjp_expv(plan, r0, times, out, info=True)
            torch.cuda.synchronize()
        finally:
            mjp.mjp_plan_destroy(plan)
        res.append(out.cpu().numpy())
        paths.append(inf[0]["path"])
        say(f"    variant {variant}: path {inf[0]['path']}, K {[i['K'] for i in inf]}")
    want = mjp.MJP_PATH_PERSISTENT_MULTIJUMP if renorm % 4 == 0 else mjp.MJP_PATH_PERSISTENT_TWOJUMP
    assert paths == [want, mjp.MJP_PATH_PERSISTENT]
    assert np.array_equal(res[0], res[1])


def test_exchange_probe_is_a_floor():
    """mjp_probe_exchange times the two-jump sweep's communication alone on
    the plan's own launch: it must take less per round than a solve's
    rounds do (which add two jumps of arithmetic to the same exchange)."""
    model = mjp.make_model(mjp.MJP_MODEL_CASCADE2, [200.0, 1.0, 0.5, 0.5], [1000, 1000])
    plan = mjp.mjp_plan_create_stencil(model, mjp.mjp_opts_default(variant=mjp.MJP_VARIANT_PERSISTENT_TWOJUMP))
    try:
        r0 = torch.zeros(10 ** 6, device="cuda")
        r0[0] = 1.0
        out = torch.empty((1, 10 ** 6), device="cuda")
        info = mjp.mjp_expv(plan, r0, [1.0], out, info=True)[0]
        assert info["path"] == mjp.MJP_PATH_PERSISTENT_TWOJUMP
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        mjp.mjp_expv(plan, r0, [1.0], out)
        ev1.record()
        torch.cuda.synchronize()
        per_round = ev0.elapsed_time(ev1) * 1e3 / ((info["K"] + 1) // 2)
        floor = mjp.mjp_probe_exchange(plan, (info["K"] + 1) // 2)
        print(f"[gpu] exchange floor {floor:.2f} us per round, solve {per_round:.2f} us per round", file=sys.stderr)
        assert 0.2 < floor < per_round
    finally:
        mjp.mjp_plan_destroy(plan)


def test_tiled_exchange_probe_is_a_floor():
    """mjp_probe_exchange2 on the tiled sweep's launch and tables (eight jumps
    per round at this size): the exchange alone must take less per round
    than a solve's rounds do."""
    model = mjp.make_model(mjp.MJP_MODEL_CASCADE2, [200.0, 1.0, 0.5, 0.5], [1000, 1000])
    plan = mjp.mjp_plan_create_stencil(model)
    try:
        r0 = torch.zeros(10 ** 6, device="cuda")
        r0[0] = 1.0
        out = torch.empty((1, 10 ** 6), device="cuda")
        info = mjp.mjp_expv(plan, r0, [1.0], out, info=True)[0]
        assert info["path"] == mjp.MJP_PATH_PERSISTENT_MULTIJUMP
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        mjp.mjp_expv(plan, r0, [1.0], out)
        ev1.record()
        torch.cuda.synchronize()
        _, jumps = mjp.mjp_probe_exchange2(plan, 10)
        assert jumps == 8
        rounds = -(-info["K"] // jumps)
        per_round = ev0.elapsed_time(ev1) * 1e3 / rounds
        floor, _ = mjp.mjp_probe_exchange2(plan, rounds)
        print(f"[gpu] tiled exchange floor {floor:.2f} us per round, solve {per_round:.2f} us per round",
              file=sys.stderr)
        assert 0.2 < floor < per_round
    finally:
        mjp.mjp_plan_destroy(plan)
