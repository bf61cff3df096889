"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds only input generation: random numbers, initial vectors, time
grids, random rate graphs and stochastic-simulation snapshot data.  It
contains none of the expansion's arithmetic (no Omega, no uniformised matrix,
no Poisson weights, no series), so both the HIP path and the FP64 oracle can
take their inputs from here without sharing any of the method.

Every generator takes an explicit integer seed and draws from numpy's Philox
counter-based bit generator, so a seed names the same data on every machine.

Workload recipes (rates, grid sizes and data designs follow the paper's
synthetic experiments, Sec. 3.1):

* birth-death (Eq. BD_def): N states, birth beta, death gamma*n, start at 0;
* two-species cascade: S1 x S2 grid, rates (k1, g1, k2, g2), start at (0, 0);
* snapshot data: independent Gillespie runs per collection time, observing the
  full state at that time (the snapshot scheme of Sec. 2.1.2), collection
  times evenly spaced as in Sec. 3.1.2 / 3.1.3.
"""
from __future__ import annotations

import numpy as np

SEED_DATA = 231205647
SEED_THETA = 231205648
SEED_MCMC = 231205649
SEED_MLP = 231205650


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(int(seed)))


# ---------------------------------------------------------------- vectors ---

def delta(n: int, at: int = 0, dtype=np.float64) -> np.ndarray:
    v = np.zeros(n, dtype=dtype)
    v[at] = 1
    return v


def random_prob(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """A dense probability vector (Dirichlet(1) draw)."""
    x = rng(seed).exponential(size=n)
    return (x / x.sum()).astype(dtype)


def log_spaced_times(n: int = 16, lo: float = 0.1, hi: float = 10.0) -> np.ndarray:
    """n log-spaced collection times in [lo, hi] (the 16-time workload)."""
    return np.array([lo * (hi / lo) ** (j / (n - 1)) for j in range(n)], dtype=np.float64)


def even_times(n: int = 20, step: float = 0.5) -> np.ndarray:
    """T_i = step * i, i = 1..n (collection times 0.5..10 as in Sec. 3.1.2)."""
    return step * np.arange(1, n + 1, dtype=np.float64)


# ------------------------------------------------------ random rate graphs ---

def random_rate_graph(n: int, seed: int, degree: int = 3, scale: float = 5.0,
                      dense: bool = False):
    """Random non-negative transition rates lambda_nm (n != m).

    Returns (row_ptr int64[n+1], col int32[nnz], rate float64[nnz]) of the
    off-diagonal rates only, rows sorted by column.  ``dense`` gives every pair
    a rate (for small dense cross-checks).
    """
    g = rng(seed)
    rows, cols, rates = [], [], []
    for r in range(n):
        if dense:
            targets = [m for m in range(n) if m != r]
        else:
            k = int(g.integers(1, degree + 1))
            targets = sorted(set(int(x) for x in g.integers(0, n, size=k)) - {r})
        for m in targets:
            rows.append(r)
            cols.append(m)
            rates.append(float(g.exponential(scale)))
    row_ptr = np.zeros(n + 1, np.int64)
    for r in rows:
        row_ptr[r + 1] += 1
    row_ptr = np.cumsum(row_ptr)
    return row_ptr, np.array(cols, np.int32), np.array(rates, np.float64)


def with_generator_diagonal(row_ptr, col, rate):
    """Insert a_nn = -sum_m lambda_nm into a rate graph, giving a generator in
    CSR (row = from-state).  This is the definition of a generator's diagonal,
    needed to hand a valid input to either side; it is not part of the
    expansion."""
    n = len(row_ptr) - 1
    out_rp = np.zeros(n + 1, np.int64)
    out_c, out_v = [], []
    for r in range(n):
        lo, hi = row_ptr[r], row_ptr[r + 1]
        ent = list(zip(col[lo:hi].tolist(), rate[lo:hi].tolist()))
        ent.append((r, -float(np.sum(rate[lo:hi]))))
        ent.sort()
        for c, v in ent:
            out_c.append(c)
            out_v.append(v)
        out_rp[r + 1] = len(out_c)
    return out_rp, np.array(out_c, np.int32), np.array(out_v, np.float64)


# ------------------------------------------------------------- theta draws ---

def theta_draws(B: int, theta_star, seed: int = SEED_THETA, decades: float = 1.0) -> np.ndarray:
    """B draws, log-uniform over ``decades`` decades centred on theta_star."""
    g = rng(seed)
    half = 0.5 * decades * np.log(10.0)
    psi = np.log(np.asarray(theta_star, np.float64))[None, :] + g.uniform(-half, half, size=(B, len(theta_star)))
    return np.exp(psi)


# --------------------------------------------------- Gillespie snapshot data --

def _gillespie_lockstep(g, n_runs: int, T: float, propensities, updates, state0):
    """Simulate n_runs independent trajectories of a reaction network up to
    time T with Gillespie's direct method (all runs advanced in lockstep),
    returning the final states.  propensities(state) -> (n_runs, R) array;
    updates is an (R, d) integer array of state changes."""
    state = np.tile(np.asarray(state0, np.int64), (n_runs, 1))
    t = np.zeros(n_runs)
    alive = np.ones(n_runs, bool)
    while alive.any():
        idx = np.nonzero(alive)[0]
        a = propensities(state[idx])
        a0 = a.sum(axis=1)
        stuck = a0 <= 0
        dt = np.where(stuck, np.inf, g.exponential(size=len(idx)) / np.where(stuck, 1.0, a0))
        t_new = t[idx] + dt
        done = t_new > T
        alive[idx[done]] = False
        go = ~done
        if not go.any():
            break
        gi = idx[go]
        t[gi] = t_new[go]
        cum = np.cumsum(a[go], axis=1)
        u = g.uniform(size=len(gi)) * a0[go]
        r = (cum < u[:, None]).sum(axis=1)
        r = np.minimum(r, a.shape[1] - 1)
        state[gi] += updates[r]
    return state


def gillespie_bd(beta: float, gamma: float, times, n_per_time: int, seed: int = SEED_DATA):
    """Birth-death snapshot data (Sec. 3.1.1): independent runs from 0,
    observed at each time.  Returns an (I, 2) array of (time index, count)."""
    g = rng(seed)
    upd = np.array([[1], [-1]], np.int64)

    def prop(s):
        n = s[:, 0].astype(np.float64)
        return np.stack([np.full_like(n, beta), gamma * n], axis=1)

    out = []
    for j, T in enumerate(times):
        fin = _gillespie_lockstep(g, n_per_time, float(T), prop, upd, [0])
        out.append(np.stack([np.full(n_per_time, j), fin[:, 0]], axis=1))
    return np.concatenate(out).astype(np.int64)


def gillespie_cascade2(theta, times, n_per_time: int, seed: int = SEED_DATA):
    """Two-species cascade snapshot data: independent runs from (0, 0),
    observed as the full pair (n1, n2) at each time.  Returns an (I, 3) array
    of (time index, n1, n2)."""
    k1, g1, k2, g2 = [float(x) for x in theta]
    g = rng(seed)
    upd = np.array([[1, 0], [-1, 0], [0, 1], [0, -1]], np.int64)

    def prop(s):
        n1 = s[:, 0].astype(np.float64)
        n2 = s[:, 1].astype(np.float64)
        return np.stack([np.full_like(n1, k1), g1 * n1, k2 * n1, g2 * n2], axis=1)

    out = []
    for j, T in enumerate(times):
        fin = _gillespie_lockstep(g, n_per_time, float(T), prop, upd, [0, 0])
        out.append(np.concatenate([np.full((n_per_time, 1), j), fin], axis=1))
    return np.concatenate(out).astype(np.int64)


def gillespie_twostate(theta, times, n_per_time: int, seed: int = SEED_DATA):
    """Two-state birth-death snapshot data (Sec. 3.1.2): independent runs from
    n_R = 0 in the active gene state, observed as n_R only (the gene state is
    hidden).  theta = (beta, gamma, lambda_act, lambda_ina).  Returns an (I, 2)
    array of (time index, n_R)."""
    beta, gamma, lact, lina = [float(x) for x in theta]
    g = rng(seed)
    # state (n_R, gene state); gene 0 = active
    upd = np.array([[1, 0], [-1, 0], [0, 1], [0, -1]], np.int64)

    def prop(s):
        r = s[:, 0].astype(np.float64)
        act = s[:, 1] == 0
        return np.stack([np.where(act, beta, 0.0), gamma * r, np.where(act, lina, 0.0), np.where(act, 0.0, lact)],
                        axis=1)

    out = []
    for j, T in enumerate(times):
        fin = _gillespie_lockstep(g, n_per_time, float(T), prop, upd, [0, 0])
        out.append(np.stack([np.full(n_per_time, j), fin[:, 0]], axis=1))
    return np.concatenate(out).astype(np.int64)


def gillespie_autoreg(theta, times, n_per_time: int, seed: int = SEED_DATA):
    """Autoregulatory gene network snapshot data (Sec. 3.1.3): independent
    runs from (n_R, n_P) = (0, 0) in the active gene state, observed as
    (n_R, n_P) (the gene state is hidden).  theta = (beta_R, beta_P, gamma_R,
    gamma_P, lambda_act, lambda_ina).  Returns (I, 3) rows (time index, n_R, n_P)."""
    bR, bP, gR, gP, lact, lina = [float(x) for x in theta]
    g = rng(seed)
    # state (n_R, n_P, gene state); binding moves one P onto the gene
    upd = np.array([[1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, -1, 1], [0, 1, -1]], np.int64)

    def prop(s):
        r = s[:, 0].astype(np.float64)
        p = s[:, 1].astype(np.float64)
        act = s[:, 2] == 0
        return np.stack([np.where(act, bR, 0.0), bP * r, gR * r, gP * p, np.where(act, lina * p, 0.0),
                         np.where(act, 0.0, lact)], axis=1)

    out = []
    for j, T in enumerate(times):
        fin = _gillespie_lockstep(g, n_per_time, float(T), prop, upd, [0, 0, 0])
        out.append(np.concatenate([np.full((n_per_time, 1), j), fin[:, :2]], axis=1))
    return np.concatenate(out).astype(np.int64)


def tally(pairs: np.ndarray) -> np.ndarray:
    """Collapse repeated observation rows into (row..., count) with a count
    column appended; rows sorted lexicographically."""
    uniq, counts = np.unique(pairs, axis=0, return_counts=True)
    return np.concatenate([uniq, counts[:, None]], axis=1).astype(np.int64)


# ------------------------------------------------------------ grid sizing ---

def grid_dims(theta, max_counts, lo: int = 50, hi: int = 200, t_max: float = 10.0) -> np.ndarray:
    """Per-draw grid sides (S1, S2) for the two-species cascade.

    Each side is the larger of twice the largest observed count of that
    species (the data-driven cutoff of Sec. 3.1.1) and mean + 8 standard
    deviations of the stationary law under the draw's rates, clamped to
    [lo, hi].  theta: (B, 4) array of (k1, g1, k2, g2).  The stationary
    moments of this affine network are upper bounds of the moments at
    t <= t_max from an empty start."""
    th = np.atleast_2d(np.asarray(theta, np.float64))
    k1, g1, k2, g2 = th[:, 0], th[:, 1], th[:, 2], th[:, 3]
    m1 = k1 / g1
    c11 = m1
    m2 = k2 * m1 / g2
    c12 = k2 * c11 / (g1 + g2)
    c22 = (k2 * m1 + g2 * m2 + 2 * k2 * c12) / (2 * g2)
    s1 = np.maximum(2 * max_counts[0], np.ceil(m1 + 8 * np.sqrt(c11)))
    s2 = np.maximum(2 * max_counts[1], np.ceil(m2 + 8 * np.sqrt(c22)))
    return np.stack([np.clip(s1, lo, hi), np.clip(s2, lo, hi)], axis=1).astype(np.int32)


def cascade_records(data: np.ndarray) -> np.ndarray:
    """(time idx, n1, n2) snapshot rows -> (time idx, x1, x2, count) records."""
    return tally(data)
