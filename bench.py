"""Benchmark of the R-MJP expansion on one MI355X.

One step = one full solve rho(0) exp(A t) of the large two-species workload:
a 1000 x 1000 grid (N = 10^6 states, 4,995,001 generator entries), rates
(k1, g1, k2, g2) = (200, 1, 0.5, 0.5), rho(0) at (0, 0), t = 1, L1 truncation
budget 1e-9 (K and L from the Poisson tails), FP32 products with FP64 weights.
The operator and rho(0) are resident in HBM before timing starts.

Prints ONE JSON line (rank 0, N = 1):
  value      solves/s of the timed variant (default: CSR operator)
  roofline   the solve kernel against the bound that sets its time.  It keeps
             the operator in registers for all K jumps and exchanges only the
             iterate between neighbouring workgroups, two jumps per
             synchronisation, so the bound is that exchange ("sync"):
             achieved = jumps/s of the solve (HIP events on the stream the
             kernel runs on), peak = jumps/s if every two-jump round took only
             the measured exchange floor (mjp_probe_exchange: the same loads,
             stores, flags and waits with no arithmetic).  The survey's
             streaming byte count (52 B per row and jump for CSR) divided by
             the solve time is reported beside it as algorithmic_GBps; it
             exceeds the HBM peak because the operator is not re-read.
  cpu_baseline  the FP64 oracle on the host on the same workload
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "expv solves/s & HBM GB/s at L1≤1e-6 vs FP64; DA-MCMC ESS/s vs plain"
HBM_PEAK_GBS = 8000.0
THETA = [200.0, 1.0, 0.5, 0.5]
S1 = S2 = 1000
T_SOLVE = 1.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def algorithmic_bytes(kind: str, n: int, nnz: int, K: int, L: int) -> float:
    """Bytes one solve must move: per jump the operator and the vector once
    (CSR: values 4 B + column 4 B per entry, row pointer 4 B, x in 4 B,
    y out 4 B per row; stencil: x in + y out), plus the Kahan pair read and
    written on each accumulated jump (16 B per row)."""
    per_jump = (8 * nnz + 12 * n) if kind == "csr" else 8 * n
    return K * per_jump + (K - L + 1) * 16 * n


KERNEL_SOURCES = ("persistent.hip", "gridsync.h")


def measured_traffic(kind: str):
    """HBM bytes per launch of the solve kernel from the committed counter
    record (profiles/), used only while the kernel source is unchanged since
    the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_expv_{kind}_N1e6.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:  # the kernel and its grid synchronisation
        h.update(open(os.path.join(ROOT, "paper_2312_05647_amd", "csrc", name), "rb").read())
    if rec.get("kernel_sources_sha256") != h.hexdigest():
        return None
    return {"bytes_per_launch": rec["hbm_bytes_per_launch"], "source": os.path.relpath(path, ROOT)}


def bench_small(torch, mjp, reps: int = 20, orc=None):
    """The two smaller expv workloads.
    C1: immigration-death on states 0..999, lambda = 500, mu = 1, t = 1,
        rho(0) at 0 (latency-bound: one short sweep of ~1900 jumps); its
        result is compared with the closed form Poisson(500 (1 - e^-1)).
    C2: cascade 300 x 300 (N = 90,000), rates (200, 1, 0.5, 0.5), rho(0) at
        (0, 0), 16 log-spaced times 0.1..10 in one sweep with 16 full-vector
        outputs (K up to ~9400); its bytes are served from cache (the vector
        pair is 0.7 MB).  With the oracle (orc) each time's L1 error against
        its independent FP64 solve is reported."""
    from scipy.stats import poisson
    from paper_2312_05647_amd import synth
    res = {}
    stream = torch.cuda.current_stream()

    def run(plan, r0, times, out):
        inf = mjp.mjp_expv(plan, r0, times, out, info=True)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            mjp.mjp_expv(plan, r0, times, out, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        return inf, ev0.elapsed_time(ev1) / 1e3 / reps

    m1 = mjp.make_model(mjp.MJP_MODEL_BD, [500.0, 1.0], [1000])
    rp, ci, va = mjp.mjp_model_csr(m1)
    plan = mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default())
    r0 = torch.zeros(1000, device="cuda")
    r0[0] = 1.0
    out = torch.empty((1, 1000), device="cuda")
    try:
        inf, sec = run(plan, r0, [1.0], out)
        exact = poisson.pmf(np.arange(1000), 500.0 * (1 - math.exp(-1.0)))
        res["C1_birth_death_N1000"] = {"us_per_solve": sec * 1e6, "jumps_per_s": inf[0]["K"] / sec, "K": inf[0]["K"],
                                       "l1_vs_closed_form": float(np.abs(out[0].double().cpu().numpy() - exact).sum())}
        log(f"[bench] C1: {sec * 1e6:.1f} us/solve, K={inf[0]['K']}")
        # the same solve for a batch of initial states delta(i) (i = 0..B-1
        # mod 1000) in one mjp_expv_batched call: one workgroup per item
        B = 4096
        r0s = torch.zeros((B, 1000), device="cuda")
        r0s[torch.arange(B), torch.arange(B) % 1000] = 1.0
        outs = torch.empty((B, 1, 1000), device="cuda")
        plans, tl = [plan] * B, [[1.0]] * B
        bi = mjp.mjp_expv_batched(plans, r0s, tl, outs, info=True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(3):
            mjp.mjp_expv_batched(plans, r0s, tl, outs, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        bwall = (time.perf_counter() - t0) / 3
        bsec = ev0.elapsed_time(ev1) / 1e3 / 3
        same = bool(torch.equal(outs[0, 0], out[0]))
        res["C1_batched_4096_initial_states"] = {
            "solves_per_s": B / bsec, "solves_per_s_wall": B / bwall, "us_per_solve": bsec * 1e6 / B,
            "speedup_vs_single_calls": sec / (bsec / B), "path": bi[0]["path"], "item0_bit_equal_single": same}
        log(f"[bench] C1 batched: {B / bsec:.0f} solves/s ({sec / (bsec / B):.0f}x single calls), item 0 equal {same}")
    finally:
        mjp.mjp_plan_destroy(plan)

    m2 = mjp.make_model(mjp.MJP_MODEL_CASCADE2, [200.0, 1.0, 0.5, 0.5], [300, 300])
    rp, ci, va = mjp.mjp_model_csr(m2)
    plan = mjp.mjp_plan_create_csr(rp, ci, va, mjp.mjp_opts_default())
    times = list(synth.log_spaced_times(16, 0.1, 10.0))
    r0 = torch.zeros(90000, device="cuda")
    r0[0] = 1.0
    out = torch.empty((16, 90000), device="cuda")
    try:
        inf, sec = run(plan, r0, times, out)
    finally:
        mjp.mjp_plan_destroy(plan)
    Kmax = max(i["K"] for i in inf)
    acc = sum(i["K"] - i["L"] + 1 for i in inf)
    ab = Kmax * (8 * len(ci) + 12 * 90000) + acc * 16 * 90000
    res["C2_cascade_300x300_16_times"] = {"ms_per_sweep": sec * 1e3, "K_max": Kmax, "jumps_per_s": Kmax / sec,
                                          "algorithmic_GBps_cache_served": ab / sec / 1e9}
    if orc is not None:
        A2 = orc.model_generator(orc.MODEL_CASCADE2, [200.0, 1.0, 0.5, 0.5], [300, 300])
        ref = orc.expv_times(A2, synth.delta(90000), times)
        l1 = np.abs(out.double().cpu().numpy() - ref).sum(axis=1)
        res["C2_cascade_300x300_16_times"]["l1_vs_fp64_oracle_per_time"] = [float(v) for v in l1]
        res["C2_cascade_300x300_16_times"]["times"] = [float(t) for t in times]
        log(f"[bench] C2 L1 vs FP64 per time: max {l1.max():.2e}")
    log(f"[bench] C2: {sec * 1e3:.2f} ms per 16-time sweep, K_max={Kmax}")
    return res


def krylov_bytes_per_step(kappa: int, n: int, nnz: int, fused: bool) -> float:
    """Bytes the Krylov step streams: per Arnoldi iteration i = 1..kappa-1 the
    product (12 B per stored entry of A^T, the gathered vector) and three
    passes that read the i earlier basis vectors (projections,
    reorthogonalisation, norm); the new vector is written by the product and
    read/written by the two later passes in the per-pass launches (8 B x 6 per
    state with the gather), but kept in LDS and written once by the fused
    step (8 B x 2); then the combination reads kappa vectors and writes one.
    The paper's modified Gram-Schmidt streams the same 24 B per state per
    earlier vector (i dependent passes, each reading q_j and reading and
    writing w), so this is also the method's own traffic, not only the
    implementation's (classical Gram-Schmidt with one reorthogonalisation)."""
    own = 2 if fused else 6
    per_i = sum(12 * nnz + 8 * n * (3 * i + own) for i in range(1, kappa))
    return per_i + 8 * n * (kappa + 1)


def bench_krylov(torch, mjp, rp, ci, va, n, reps: int = 3):
    """Krylov propagator (Method #5) on the same N = 10^6 solve, FP64: the
    paper's step (dt_factor 2) and a converged one (dt_factor 0.5) with the
    default per-pass launches, and the paper's step as one cooperative
    launch per step (the fused variant) for comparison."""
    res = {}
    r0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    r0[0] = 1.0
    out = torch.empty((1, n), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    for f, variant in ((2.0, mjp.MJP_KRYLOV_AUTO), (0.5, mjp.MJP_KRYLOV_AUTO), (2.0, mjp.MJP_KRYLOV_FUSED)):
        h = mjp.mjp_krylov_create(rp, ci, va, mjp.mjp_krylov_opts_default(dt_factor=f, variant=variant))
        try:
            info = mjp.mjp_krylov_expv(h, r0, [T_SOLVE], out, stream=stream)
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            for _ in range(reps):
                mjp.mjp_krylov_expv(h, r0, [T_SOLVE], out, stream=stream)
            ev1.record(stream)
            torch.cuda.synchronize()
        finally:
            mjp.mjp_krylov_destroy(h)
        sec = ev0.elapsed_time(ev1) / 1e3 / reps
        fused = bool(info["fused"])
        ab = info["steps"] * krylov_bytes_per_step(info["kappa"], n, len(ci), fused)
        key = f"dt_factor_{f:g}" + ("" if variant == mjp.MJP_KRYLOV_AUTO else "_fused_step")
        res[key] = {"ms_per_solve": sec * 1e3, "steps": info["steps"], "kappa": info["kappa"],
                    "fused_step": fused, "streamed_GBps": ab / sec / 1e9,
                    "frac_of_hbm_peak": ab / sec / 1e9 / HBM_PEAK_GBS, "result": out[0].cpu().numpy()}
        log(f"[bench] krylov f={f} fused={fused}: {sec * 1e3:.2f} ms/solve, {info['steps']} steps, "
            f"{ab / sec / 1e9:.0f} GB/s")
    return res


def rk4_bytes_per_step(n: int, nnz: int) -> float:
    """Bytes the RK4 step streams: four products, each reading every stored
    entry of the merged A^T once (8 B rate, 4 B source, 1 B channel); per
    state, stage 1 reads x and writes the next input and the weighted sum
    (24 B), stages 2 and 3 read their input and x, write the next input and
    read/write the sum (40 B each), stage 4 reads its input, x and the sum
    and writes the new x (32 B): 136 B per state."""
    return 4 * 13 * nnz + 136 * n


def bench_rk4(torch, mjp, rp, ci, va, n, reps: int = 3):
    """Runge-Kutta propagator (Method #4) on the same N = 10^6 solve, FP64,
    with the paper's step bound (dt_factor 1): the generator given as one
    CSR channel, and the stencil form (the model's four reactions, entries
    formed in the kernel: only the 136 B per state of the vectors stream)."""
    r0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    r0[0] = 1.0
    stream = torch.cuda.current_stream()

    def run(h):
        out = torch.empty((1, n), dtype=torch.float64, device="cuda")
        try:
            info = mjp.mjp_rk4_expv(h, r0, [T_SOLVE], out, stream=stream)
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            for _ in range(reps):
                mjp.mjp_rk4_expv(h, r0, [T_SOLVE], out, stream=stream)
            ev1.record(stream)
            torch.cuda.synchronize()
        finally:
            mjp.mjp_rk4_destroy(h)
        return info, ev0.elapsed_time(ev1) / 1e3 / reps, out

    opts = mjp.mjp_rk4_opts_default(dt_factor=1.0)
    info, sec, out = run(mjp.mjp_rk4_create([(rp, ci, va)], opts))
    ab = info["steps"] * rk4_bytes_per_step(n, len(ci))
    log(f"[bench] rk4 f=1: {sec * 1e3:.2f} ms/solve, {info['steps']} steps, {ab / sec / 1e9:.0f} GB/s")
    sinfo, ssec, sout = run(mjp.mjp_rk4_create_stencil(mjp.make_model(mjp.MJP_MODEL_CASCADE2, THETA, [S1, S2]), opts))
    sab = sinfo["steps"] * rk4_bytes_per_step(n, 0)
    log(f"[bench] rk4 stencil f=1: {ssec * 1e3:.2f} ms/solve, {sinfo['steps']} steps, {sab / ssec / 1e9:.0f} GB/s")
    return {"ms_per_solve": sec * 1e3, "steps": info["steps"], "dt_factor": 1.0,
            "streamed_GBps": ab / sec / 1e9, "frac_of_hbm_peak": ab / sec / 1e9 / HBM_PEAK_GBS,
            "stencil": {"ms_per_solve": ssec * 1e3, "steps": sinfo["steps"], "streamed_GBps": sab / ssec / 1e9,
                        "frac_of_hbm_peak": sab / ssec / 1e9 / HBM_PEAK_GBS,
                        "l1_vs_csr_form": float((sout[0] - out[0]).abs().sum())},
            "result": out[0].cpu().numpy()}


def bench_jmjp(torch, mjp, chains: int = 512, steps: int = 300):
    """J-MJP (Method #2: Gibbs over rates and jump counts) against plain MH
    on the marginal likelihood (R-MJP) for the birth-death posterior of
    (log beta, log gamma): data 10 times 0.5..5 x 30 snapshots from
    (50, 1); both start from the same draws near the posterior and share the
    random-walk covariance (posterior covariance x 2.38^2/2).  Both run every
    step on the device (mjp_sampler_*, mjp_jmjp_*)."""
    from paper_2312_05647_amd import jmjp, sampler, synth
    beta, gamma = 50.0, 1.0
    T = np.linspace(0.5, 5.0, 10)
    data = synth.gillespie_bd(beta, gamma, T, 30, seed=synth.SEED_DATA)
    recs = np.array([[j, n, 0, c] for j, n, c in synth.tally(data)], np.int32)
    N = max(2 * int(data[:, 1].max()), 120)
    g = synth.rng(12)
    center = np.log([beta, gamma])
    cov = np.diag([0.004, 0.004])
    psi0 = torch.as_tensor(g.multivariate_normal(center, cov, size=chains), device="cuda")
    mh_post = sampler.Posterior(mjp.MJP_MODEL_BD, T, recs, (N, 1), n_par=2)
    # posterior covariance from a short MH pilot, shared by both samplers
    pilot, _ = sampler.run_device(mh_post, psi0, cov * 2.38 ** 2 / 2, 200, seed=13)
    Z = np.cov(pilot[100:].reshape(-1, 2).T) * 2.38 ** 2 / 2
    psi1 = torch.as_tensor(pilot[-1], device="cuda")
    s_mh, st_mh = sampler.run_device(mh_post, psi1, Z, steps, seed=14)
    post = jmjp.JumpPosterior(mjp.MJP_MODEL_BD, T, recs, (N, 1), n_par=2)
    s_j, st_j = jmjp.run_jmjp_device(post, psi1, Z, steps, seed=15)
    e_mh, e_j = sampler.ess(s_mh), sampler.ess(s_j)
    res = {"workload": f"birth-death posterior, {post.I} snapshots, {chains} chains x {steps} steps per sampler",
           "ess_per_s_mh_rmjp": float(e_mh.min() / st_mh.seconds), "ess_per_s_jmjp": float(e_j.min() / st_j.seconds),
           "ess_per_step_mh_rmjp": float(e_mh.min() / steps), "ess_per_step_jmjp": float(e_j.min() / steps),
           "seconds_mh": st_mh.seconds, "seconds_jmjp": st_j.seconds,
           "jmjp_theta_accept": st_j.theta_accepted / (steps * chains), "jmjp_k_accept": st_j.k_accept_rate,
           "mh_accept": st_mh.accepted / (steps * chains),
           "posterior_mean_mh": s_mh.reshape(-1, 2).mean(0).tolist(),
           "posterior_mean_jmjp": s_j.reshape(-1, 2).mean(0).tolist()}
    log(f"[bench] J-MJP: ESS/s {res['ess_per_s_jmjp']:.1f} vs MH on R-MJP {res['ess_per_s_mh_rmjp']:.1f} "
        f"(ESS/step {res['ess_per_step_jmjp']:.3f} vs {res['ess_per_step_mh_rmjp']:.3f})")
    return res


MLP_FLOP_PER_SAMPLE_EPOCH = 2 * ((4 * 256 + 256 * 256 * 2 + 256)        # forward
                                 + (256 * 256 * 2 + 256)                # data gradients (layers 2-4)
                                 + (4 * 256 + 256 * 256 * 2 + 256))     # weight gradients
MFMA_BF16_PEAK_TFLOPS = 2500.0


def bench_surrogate(torch, mjp, n: int = 16384, epochs: int = 60):
    """Training of the 4-256-256-256-1 surrogate (BF16 MFMA GEMMs, FP32
    accumulate, Adam) on n synthetic standardised inputs with a smooth target,
    at the delayed-acceptance leg's batch (1024) and at 4096; achieved
    TFLOP/s from 792,064 FLOP per sample and epoch (forward, data and weight
    gradients) against the 2.5 PFLOP/s dense BF16 peak."""
    from paper_2312_05647_amd import synth
    g = synth.rng(41)
    x = torch.as_tensor(g.standard_normal((n, 4)), dtype=torch.float32, device="cuda").contiguous()
    xs = x.double()
    y = (-(xs ** 2).sum(1) + 0.3 * xs[:, 0] * xs[:, 1]).float().contiguous()
    res = {}
    for batch in (1024, 4096):
        h = mjp.mjp_surrogate_create(4, 256, 3, seed=0)
        try:
            cfg = mjp.mjp_train_cfg_default(epochs=epochs, batch=batch, lr=2e-3, seed=0)
            mjp.mjp_surrogate_train(h, x, y, mjp.mjp_train_cfg_default(epochs=1, batch=batch, lr=2e-3, seed=0))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            losses = mjp.mjp_surrogate_train(h, x, y, cfg)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
        finally:
            mjp.mjp_surrogate_destroy(h)
        tf = MLP_FLOP_PER_SAMPLE_EPOCH * n * epochs / sec / 1e12
        res[f"batch_{batch}"] = {"seconds": sec, "samples_per_s": n * epochs / sec, "achieved_TFLOPs": tf,
                                 "frac_of_bf16_mfma_peak": tf / MFMA_BF16_PEAK_TFLOPS,
                                 "loss_first_last": [float(losses[0]), float(losses[-1])]}
        log(f"[bench] surrogate training batch {batch}: {sec:.3f} s, {tf:.2f} TFLOP/s "
            f"({tf / MFMA_BF16_PEAK_TFLOPS:.4%} of peak)")
    return {"workload": f"MLP 4-256-256-256-1, {n} samples x {epochs} epochs", **res}


def bench_loglik(torch, mjp, reps: int = 3):
    """Batched log-likelihoods: 4096 draws log-uniform over a decade around
    (50, 1, 0.5, 0.5), 20 collection times 0.5..10 with 50 snapshots each,
    per-draw grids of 50..200 per side, one persistent launch per batch."""
    import ctypes
    from paper_2312_05647_amd import synth
    theta_star = [50.0, 1.0, 0.5, 0.5]
    T = synth.even_times(20, 0.5)
    data = synth.gillespie_cascade2(theta_star, T, 50, seed=synth.SEED_DATA)
    recs = synth.cascade_records(data)
    theta = synth.theta_draws(4096, theta_star, seed=synth.SEED_THETA)
    dims = synth.grid_dims(theta, (int(data[:, 1].max()), int(data[:, 2].max())))
    B = len(theta)
    th = torch.as_tensor(theta, device="cuda")
    dm = torch.as_tensor(dims, device="cuda")
    out = torch.empty(B, dtype=torch.float64, device="cuda")
    info = torch.zeros(B * ctypes.sizeof(mjp.mjp_info), dtype=torch.uint8, device="cuda")
    obs = mjp.make_obs(T, recs, (0, 0))
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed():
        ev0.record(stream)
        for _ in range(reps):
            mjp.mjp_loglik(1, th, dm, obs, out, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / 1e3 / reps

    # default launch shapes
    mjp.mjp_loglik(1, th, dm, obs, out, info=info, stream=stream)
    torch.cuda.synchronize()
    sec = timed()
    raw = info.cpu().numpy().tobytes()
    sz = ctypes.sizeof(mjp.mjp_info)
    infos = [mjp.mjp_info.from_buffer_copy(raw[i * sz:(i + 1) * sz]) for i in range(B)]
    K = np.array([i.K for i in infos], np.float64)
    vals = out.cpu().numpy()
    reasons = {"out_of_grid": 0, "fp32_underflow_at_observed_state": 0, "k_cap": 0, "other": 0}
    for v, i in zip(vals, infos):
        if np.isfinite(v):
            continue
        if i.flags & mjp.MJP_FLAG_K_LIMIT:
            reasons["k_cap"] += 1
        elif i.flags & mjp.MJP_FLAG_OUT_OF_GRID:
            reasons["out_of_grid"] += 1
        elif i.flags & mjp.MJP_FLAG_UNDERFLOW_OBS:
            reasons["fp32_underflow_at_observed_state"] += 1
        else:
            reasons["other"] += 1
    cells = float(np.sum((K + 1) * dims[:, 0] * dims[:, 1]))
    default_shapes = mjp.mjp_loglik_get_shapes(1, len(recs))
    log(f"[bench] loglik batch: {sec * 1e3:.1f} ms for {B} draws, {B / sec:.0f} loglik/s (default shapes)")
    # autotuner: time every eligible launch shape per size class on this batch
    rep = mjp.mjp_loglik_tune(1, th, dm, obs, out, reps=1, stream=stream)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(reps):
        mjp.mjp_loglik(1, th, dm, obs, out, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    sec_t = ev0.elapsed_time(ev1) / 1e3 / reps
    shapes = mjp.mjp_loglik_shapes()
    log(f"[bench] loglik batch tuned: {sec_t * 1e3:.1f} ms, shapes {rep['chosen']} (items per class {rep['items']})")
    return {"workload": "4096 cascade draws, grids 148..200 per side, 20 times x 50 snapshots",
            "loglik_per_s": B / sec_t, "ms_per_batch": sec_t * 1e3,
            "cell_updates_per_s": cells / sec_t,
            "lds_equiv_GBps": 8 * cells / sec_t / 1e9,
            "finite_fraction": float(np.isfinite(vals).mean()),
            "minus_inf_reasons": reasons,
            "ms_per_batch_default_shapes": sec * 1e3,
            "tuner": {"items_per_class": rep["items"],
                      "default": [f"{shapes[i]['threads']}x{shapes[i]['cells']}" for i in default_shapes],
                      "chosen": [f"{shapes[i]['threads']}x{shapes[i]['cells']}" for i in rep["chosen"]],
                      "ms_per_class_shape": {f"class{c}": {f"{shapes[i]['threads']}x{shapes[i]['cells']}": v
                                                           for i, v in enumerate(rep["ms"][c][:len(shapes)]) if v >= 0}
                                             for c in range(mjp.MJP_LL_CLASSES) if rep["items"][c] > 0}}}


def bench_da(torch, mjp, chains: int = 256, steps: int = 60, n_train: int = 4096, pilot_chains: int = 128,
             pilot_steps: int = 30):
    """Delayed-acceptance vs plain Metropolis-Hastings on the posterior of
    the cascade's four log-rates with config-2 truth (200, 1, 0.5, 0.5) on
    the 300 x 300 grid (N = 90,000 states: every exact log-likelihood runs
    in a cluster of workgroups): data 20 times 0.5..10 x 50 snapshots.
    A pilot MH run (pilot_chains from independent starts near the truth,
    the SI's small initial covariance, then one covariance estimate) gives
    the proposal covariance (pooled covariance x 2.38^2/4) and a Gaussian
    approximation of the posterior; both samplers then run `chains` chains
    from the same independent draws of that Gaussian with the same
    covariance.  The surrogate is trained on n_train exact evaluations at
    draws from the Gaussian with 3x the pilot's standard deviations.  Every
    step of every chain runs on the device (mjp_sampler_*: Philox draws,
    the screen, the masked exact likelihood, the accept step)."""
    from paper_2312_05647_amd import sampler, synth
    theta_star = np.array([200.0, 1.0, 0.5, 0.5])
    T = synth.even_times(20, 0.5)
    data = synth.gillespie_cascade2(theta_star, T, 50, seed=synth.SEED_DATA)
    recs = synth.cascade_records(data)
    dims = (300, 300)
    post = sampler.Posterior(mjp.MJP_MODEL_CASCADE2, T, recs, dims)
    g = synth.rng(synth.SEED_MCMC)
    t0 = time.perf_counter()
    psi0 = torch.as_tensor(np.log(theta_star) + 0.01 * g.standard_normal((pilot_chains, 4)), device="cuda")
    Z0 = 2e-5 * np.eye(4)
    smp, _ = sampler.run_device(post, psi0, Z0, pilot_steps, seed=synth.SEED_MCMC + 1,
                                progress=lambda h: log(f"[bench] DA pilot 1: {h}"))
    half = pilot_steps // 2
    smp2, _ = sampler.run_device(post, torch.as_tensor(smp[-1], device="cuda"),
                                 2.38 ** 2 / 4 * np.cov(smp[half:].reshape(-1, 4).T), pilot_steps,
                                 seed=synth.SEED_MCMC + 2, progress=lambda h: log(f"[bench] DA pilot 2: {h}"))
    pilot = smp2[half:].reshape(-1, 4)
    pm, pc = pilot.mean(0), np.cov(pilot.T)
    Z = 2.38 ** 2 / 4 * pc
    t_pilot = time.perf_counter() - t0
    starts = torch.as_tensor(g.multivariate_normal(pm, pc, size=chains), device="cuda")
    pts = g.multivariate_normal(pm, 9.0 * pc, size=n_train)
    t0 = time.perf_counter()
    parts = []
    for i in range(0, n_train, 4096):
        parts.append(post.loglik(torch.as_tensor(pts[i:i + 4096], device="cuda")).cpu())
        log(f"[bench] DA leg: {i + len(parts[-1])}/{n_train} training evaluations, {time.perf_counter() - t0:.1f} s")
    ll = torch.cat(parts).numpy()
    t_data = time.perf_counter() - t0
    ok = np.isfinite(ll)
    screen, losses, t_train = sampler.train_surrogate(pts[ok], ll[ok], epochs=60, batch=1024, seed=synth.SEED_MLP)
    res = {}
    try:
        def prog(name):
            return lambda h: log(f"[bench] DA leg {name}: step {h}/{steps}")
        # every step on the device (Philox draws, screen, masked exact likelihood, accept)
        for name, run in (("plain_mh", lambda: sampler.run_device(post, starts, Z, steps, seed=synth.SEED_MCMC + 3,
                                                                  progress=prog("mh"))),
                          ("delayed_acceptance",
                           lambda: sampler.run_device(post, starts, Z, steps, seed=synth.SEED_MCMC + 4, screen=screen,
                                                      progress=prog("da")))):
            smp, st = run()
            e = sampler.ess(smp)
            flat = smp.reshape(-1, smp.shape[2])
            var = flat.var(0)
            res[name] = {"ess_min": float(e.min()), "ess_per_s": float(e.min() / st.seconds),
                         "seconds": st.seconds, "exact_evals": st.exact_evals,
                         "accept_rate": st.accepted / (steps * chains),
                         "stage1_accept_rate": (st.stage1_accepted / (steps * chains)) if name != "plain_mh" else None,
                         "mean_log_theta": flat.mean(0).tolist(), "var_log_theta": var.tolist(),
                         "mcse_mean": np.sqrt(var / e).tolist(),
                         # the variance estimate's standard error: var sqrt(2 / ESS) (Gaussian fourth moment)
                         "mcse_var": (var * np.sqrt(2.0 / e)).tolist()}
            log(f"[bench] DA leg {name}: ESS/s {res[name]['ess_per_s']:.1f}, {st.seconds:.2f} s, exact {st.exact_evals}")
    finally:
        mjp.mjp_surrogate_destroy(screen.h)
    mh, da = res["plain_mh"], res["delayed_acceptance"]
    zm = np.abs(np.array(mh["mean_log_theta"]) - np.array(da["mean_log_theta"])) / np.hypot(mh["mcse_mean"], da["mcse_mean"])
    zv = np.abs(np.array(mh["var_log_theta"]) - np.array(da["var_log_theta"])) / np.hypot(mh["mcse_var"], da["mcse_var"])
    return {"workload": f"cascade posterior, truth (200, 1, 0.5, 0.5), grid 300x300 (N=90,000), {len(recs)} records, "
                        f"{chains} chains x {steps} steps per sampler from independent starts, surrogate "
                        f"4-256-256-256-1 on {int(ok.sum())} exact evaluations",
            "ess_per_s_ratio_da_over_mh": da["ess_per_s"] / mh["ess_per_s"],
            "mean_diff_in_mcse_max": float(zm.max()), "var_diff_in_mcse_max": float(zv.max()),
            "pilot_s": t_pilot, "train_data_s": t_data, "train_s": t_train,
            "train_loss_first_last": [float(losses[0]), float(losses[-1])],
            "ess_per_s_da_incl_training": da["ess_min"] / (da["seconds"] + t_data + t_train),
            **res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kind", choices=["csr", "stencil"], default="csr")
    ap.add_argument("--variant", type=int, default=0, help="0 auto, 1 stepwise, 2 persistent")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--part", choices=["all", "loglik", "da", "small", "krylov", "rk4", "jmjp", "surrogate"], default="all",
                    help="run only one secondary leg (for profiling)")
    ap.add_argument("--da-chains", type=int, default=256)
    ap.add_argument("--da-steps", type=int, default=60)
    ap.add_argument("--da-train", type=int, default=4096)
    ap.add_argument("--log-maps", metavar="FILE",
                    help="write this process's memory map to FILE at exit (to place a crash address in a library)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2312_05647_amd import mjp

    if args.log_maps:
        import atexit

        def write_maps(path=args.log_maps):
            with open("/proc/self/maps") as f, open(path, "w") as g:
                g.write(f.read())
        atexit.register(write_maps)

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4, "copies": 3}))
        return
    if args.part == "loglik":
        print(json.dumps({"loglik_batch": bench_loglik(torch, mjp)}))
        return
    if args.part == "da":
        print(json.dumps({"da_mcmc": bench_da(torch, mjp, args.da_chains, args.da_steps, args.da_train)}))
        return
    if args.part == "small":
        print(json.dumps({"small_configs": bench_small(torch, mjp)}))
        return
    if args.part == "krylov":
        rp, ci, va = mjp.mjp_model_csr(mjp.make_model(mjp.MJP_MODEL_CASCADE2, THETA, [S1, S2]))
        kr = bench_krylov(torch, mjp, rp, ci, va, S1 * S2)
        print(json.dumps({"krylov_method5": {k: {kk: vv for kk, vv in v.items() if kk != "result"}
                                             for k, v in kr.items()}}))
        return

    if args.part == "surrogate":
        print(json.dumps({"surrogate_training": bench_surrogate(torch, mjp)}))
        return
    if args.part == "jmjp":
        print(json.dumps({"jmjp_method2": bench_jmjp(torch, mjp)}))
        return
    if args.part == "rk4":
        rp, ci, va = mjp.mjp_model_csr(mjp.make_model(mjp.MJP_MODEL_CASCADE2, THETA, [S1, S2]))
        r = bench_rk4(torch, mjp, rp, ci, va, S1 * S2)
        print(json.dumps({"rk4_method4": {k: v for k, v in r.items() if k != "result"}}))
        return

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = S1 * S2
    model = mjp.make_model(mjp.MJP_MODEL_CASCADE2, THETA, [S1, S2])
    opts = mjp.mjp_opts_default(variant=args.variant)
    rp, ci, va = mjp.mjp_model_csr(model)
    nnz = len(ci)

    def make_plan(kind):
        return mjp.mjp_plan_create_csr(rp, ci, va, opts) if kind == "csr" else mjp.mjp_plan_create_stencil(model, opts)

    rho0 = torch.zeros(n, dtype=torch.float32, device=dev)
    rho0[0] = 1.0
    out = torch.empty((1, n), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def time_solves(plan, steps, warmup):
        info = mjp.mjp_expv(plan, rho0, [T_SOLVE], out, info=True)[0]   # also a warm-up
        for _ in range(warmup):
            mjp.mjp_expv(plan, rho0, [T_SOLVE], out, stream=stream)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(steps):
            mjp.mjp_expv(plan, rho0, [T_SOLVE], out, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return info, ev0.elapsed_time(ev1) / 1e3 / steps, wall

    def exchange_floor(plan, K, path):
        """(rounds per solve, floor us per round, jumps per round) of a sweep
        with several jumps per synchronisation (the tiled or the two-jump
        kernel); None where the plan's sweep synchronises every jump."""
        if path not in (mjp.MJP_PATH_PERSISTENT_TWOJUMP, mjp.MJP_PATH_PERSISTENT_MULTIJUMP):
            return None
        _, jumps = mjp.mjp_probe_exchange2(plan, 50, stream=stream)
        rounds = -(-K // jumps)
        floor, _ = mjp.mjp_probe_exchange2(plan, rounds, stream=stream)
        return rounds, floor, jumps

    log(f"[bench] plan {args.kind} N={n} nnz={nnz}")
    plan = make_plan(args.kind)
    info, dev_s, wall = time_solves(plan, args.steps, args.warmup)
    got = out[0].double().cpu().numpy()
    xfloor = exchange_floor(plan, info["K"], info.get("path"))
    mjp.mjp_plan_destroy(plan)
    K, L = info["K"], info["L"]
    ab = algorithmic_bytes(args.kind, n, nnz, K, L)
    achieved = ab / dev_s / 1e9
    log(f"[bench] {args.kind}: {dev_s * 1e3:.3f} ms/solve (device events), wall {wall / args.steps * 1e3:.3f} ms, "
        f"K={K} L={L}, {achieved:.0f} GB/s algorithmic")

    traffic = measured_traffic(args.kind)
    if xfloor is not None:
        rounds, floor_us, jumps = xfloor
        meas_us = dev_s * 1e6 / rounds
        peak = jumps / (floor_us * 1e-6)  # the jump rate if the arithmetic took no time
        roof = {"bound": "sync", "achieved": K / dev_s, "peak": peak, "unit": "jumps/s",
                "frac": (K / dev_s) / peak,
                "kernel": f"one solve (all K jumps, weighted accumulation, lumping), {jumps} jumps per "
                          f"neighbour exchange" + (" on 2-D tiles" if jumps > 2 else ""),
                "jumps_per_sync": jumps, "rounds_per_solve": rounds, "us_per_round_measured": meas_us,
                "us_per_round_exchange_floor": floor_us,
                "us_per_round_arithmetic": meas_us - floor_us,
                "floor_source": "mjp_probe_exchange2: the same device-scope halo loads, own-row stores, drain, "
                                "flags and waits on the same launch and tables, no arithmetic"}
        log(f"[bench] {args.kind}: {meas_us:.2f} us per {jumps}-jump round, exchange floor {floor_us:.2f} us "
            f"({roof['frac']:.2f})")
    else:
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "kernel": "one solve, stepwise launches"}
    roof.update({"traffic": traffic["bytes_per_launch"] if traffic else None,
                 "traffic_source": traffic["source"] if traffic else "no counter record for the current kernel source",
                 "traffic_frac_of_hbm_peak": (traffic["bytes_per_launch"] / dev_s / 1e9 / HBM_PEAK_GBS) if traffic else None,
                 "algorithmic_bytes_per_solve": ab, "algorithmic_GBps": achieved,
                 "ms_per_solve_device": dev_s * 1e3})
    result = {
        "metric": METRIC,
        "value": 1.0 / (wall / args.steps),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"two-species cascade {S1}x{S2} (N=1e6, nnz={nnz}), rates {THETA}, rho0=delta(0,0), "
                               f"t={T_SOLVE}, tol=1e-9, {args.kind.upper()} FP32 operator",
                   "operator": args.kind, "variant": args.variant, "K": K, "L": L,
                   "omega": info["omega"], "global_batch": 1, "parallelism": "single GPU"},
        "roofline": roof,
    }

    if not args.no_extra:
        other = "stencil" if args.kind == "csr" else "csr"
        plan = make_plan(other)
        info2, dev2, wall2 = time_solves(plan, max(3, args.steps // 2), 1)
        xf2 = exchange_floor(plan, info2["K"], info2.get("path"))
        mjp.mjp_plan_destroy(plan)
        ab2 = algorithmic_bytes(other, n, nnz, info2["K"], info2["L"])
        result[f"{other}_variant"] = {"solves_per_s": 1.0 / (wall2 / max(3, args.steps // 2)),
                                      "ms_per_solve_device": dev2 * 1e3,
                                      "algorithmic_GBps": ab2 / dev2 / 1e9,
                                      "algorithmic_frac_of_hbm_peak": ab2 / dev2 / 1e9 / HBM_PEAK_GBS}
        if xf2 is not None:
            r2, f2, j2 = xf2
            result[f"{other}_variant"].update({"jumps_per_sync": j2, "us_per_round_measured": dev2 * 1e6 / r2,
                                               "us_per_round_exchange_floor": f2,
                                               "sync_frac": (info2["K"] / dev2) / (j2 / (f2 * 1e-6))})
        log(f"[bench] {other}: {dev2 * 1e3:.3f} ms/solve")

    kry = None
    if not args.no_extra:
        kry = bench_krylov(torch, mjp, rp, ci, va, n)
        result["krylov_method5"] = {k: {kk: vv for kk, vv in v.items() if kk != "result"} for k, v in kry.items()}
        for k, v in kry.items():  # accuracy against the FP32 R-MJP result (its own L1 vs FP64 is ~3e-7)
            result["krylov_method5"][k]["l1_vs_rmjp_gpu"] = float(np.abs(v["result"] - got).sum())
        rk = bench_rk4(torch, mjp, rp, ci, va, n)
        result["rk4_method4"] = {k: v for k, v in rk.items() if k != "result"}
        result["rk4_method4"]["l1_vs_rmjp_gpu"] = float(np.abs(rk["result"] - got).sum())
        orc = None
        if not args.no_cpu:
            import oracle as orc
            orc.build(force=False)
        result["small_configs"] = bench_small(torch, mjp, orc=orc)
        result["loglik_batch"] = bench_loglik(torch, mjp)
        result["da_mcmc"] = bench_da(torch, mjp, args.da_chains, args.da_steps, args.da_train)
        result["jmjp_method2"] = bench_jmjp(torch, mjp)
        result["surrogate_training"] = bench_surrogate(torch, mjp)

    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        A = oracle.model_generator(1, THETA, [S1, S2])
        r0 = np.zeros(n)
        r0[0] = 1.0
        eps_r = opts.tol / 4
        log(f"[bench] oracle on {oracle.num_threads()} threads")
        t0 = time.perf_counter()
        solves = 0
        ref = None
        while True:
            ref, oinfo = oracle.expv(A, r0, T_SOLVE, eps_right=eps_r)
            solves += 1
            if time.perf_counter() - t0 > 10.0 or solves >= 3:
                break
        cpu_s = (time.perf_counter() - t0) / solves
        result["cpu_baseline"] = {"value": 1.0 / cpu_s, "unit": "solves/s", "cores": oracle.num_threads(),
                                  "cpu_model": cpu_model(), "kind": "oracle",
                                  "sample": f"{solves} full FP64 solve(s) of the same workload (K={oinfo['K']}, "
                                            f"right tail {eps_r:g}), OpenMP over rows"}
        l1 = float(np.abs(got - ref).sum())
        result["parity"] = {"l1_vs_fp64_oracle": l1, "linf": float(np.abs(got - ref).max()), "bar": 1e-6}
        if kry:
            for k, v in kry.items():
                result["krylov_method5"][k]["l1_vs_fp64_oracle"] = float(np.abs(v["result"] - ref).sum())
        log(f"[bench] oracle {cpu_s:.2f} s/solve; GPU L1 vs oracle {l1:.3e}")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
