"""FP64 CPU oracle for the R-MJP expansion: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never links, loads
or calls it, and it shares no code with the HIP path (the only thing both sides
see is the seeded input generator module, which holds none of the method's
arithmetic).

What each function follows (Pessoa, Schweiger, Presse, arXiv 2312.05647):

* ``model_generator`` -- Eq. A_def with the birth-death rates of Eq. BD_def and
  the two-species cascade rates (first coordinate fastest, as in the paper's
  multi-index state linearisation, Sec. 3.1.2).
* ``pick_K`` / ``weights`` -- the Poisson weights of Eq. ME_uniform and the
  cutoff of Sec. 2.2.3 (paper rule k* = W + 6 sqrt W), formed in log space.
* ``expv`` -- Algorithm 2 (R-MJP), including the residual lumping of its last
  line.
* ``loglik`` -- the snapshot likelihood p(s^i | theta) = rho(T^i)_{s^i}
  (Sec. 2.1.2), one independent solve per collection time.
* ``oracle.mlp`` -- an FP64 reference of the surrogate network (forward,
  backward, and the Adam update ``adam_step`` of Kingma and Ba, Algorithm 1,
  with decoupled weight decay), used to check the GPU training kernels (the
  surrogate itself is not in the paper).
* ``oracle.krylov`` -- the Krylov-subspace propagator (Method #5, Algorithm
  ArnoldiKrylov, Eq. Krylov_expansion) in numpy FP64.
* ``oracle.rk4`` -- the fourth-order Runge-Kutta propagator (Method #4, Eqs.
  RKstep / RKintermediate) with time-dependent rates, numpy FP64.
* ``oracle.jmjp`` -- J-MJP (Method #2): the state probabilities given the
  jump counts (its Algorithm) and the jump-count conditional, FP64.

Parity status: every function above is pinned by ``tests/test_oracle_*.py``
against closed forms, library routines (``scipy.stats.poisson``,
``scipy.linalg.expm``) or brute force; none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mjp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_mjp_oracle.so")

MODEL_BD = 0
MODEL_CASCADE2 = 1
MODEL_TWOSTATE = 2
MODEL_AUTOREG = 3
K_TOL = 0
K_PAPER = 1


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Info(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("W", ctypes.c_double),
                ("eps_right", ctypes.c_double), ("residual", ctypes.c_double),
                ("mass_in", ctypes.c_double), ("mass_out", ctypes.c_double),
                ("K", ctypes.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_model_size.argtypes = [ctypes.c_int, P, P, P]
        L.orc_model_size.restype = ctypes.c_int
        L.orc_model_generator.argtypes = [ctypes.c_int, P, P, ctypes.c_int, P, P, P]
        L.orc_model_generator.restype = ctypes.c_int64
        L.orc_poisson_logpmf.argtypes = [ctypes.c_int64, ctypes.c_double]
        L.orc_poisson_logpmf.restype = ctypes.c_double
        L.orc_pick_K.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double, P]
        L.orc_pick_K.restype = ctypes.c_int64
        L.orc_weights.argtypes = [ctypes.c_double, ctypes.c_int64, P]
        L.orc_weights.restype = ctypes.c_double
        L.orc_expv.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int, ctypes.c_double, ctypes.c_int, P, P]
        L.orc_expv.restype = ctypes.c_int
        L.orc_jump.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double, P, P]
        L.orc_jump.restype = ctypes.c_int
        L.orc_loglik.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_int32, P, ctypes.c_int32, P,
                                 ctypes.c_double, ctypes.c_int, ctypes.c_double, P]
        L.orc_loglik.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class CSR:
    """Generator A in CSR form, row = from-state (the paper's a_nm)."""
    row_ptr: np.ndarray   # int64[n+1]
    col: np.ndarray       # int32[nnz]
    val: np.ndarray       # float64[nnz]

    @property
    def n(self) -> int:
        return len(self.row_ptr) - 1

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @staticmethod
    def from_arrays(row_ptr, col, val) -> "CSR":
        return CSR(np.ascontiguousarray(row_ptr, dtype=np.int64),
                   np.ascontiguousarray(col, dtype=np.int32),
                   np.ascontiguousarray(val, dtype=np.float64))

    def dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        for r in range(self.n):
            for e in range(self.row_ptr[r], self.row_ptr[r + 1]):
                d[r, self.col[e]] += self.val[e]
        return d


def model_generator(model: int, theta, dims, leaky: bool = False) -> CSR:
    dims_a = np.ascontiguousarray(list(dims) + [0] * (2 - len(dims)), dtype=np.int32)
    th = np.ascontiguousarray(list(theta) + [0.0] * (8 - len(theta)), dtype=np.float64)
    n = np.zeros(1, np.int64)
    cap = np.zeros(1, np.int64)
    if lib().orc_model_size(model, _p(dims_a), _p(n), _p(cap)) != 0:
        raise ValueError("bad model or dims")
    rp = np.zeros(int(n[0]) + 1, np.int64)
    ci = np.zeros(int(cap[0]), np.int32)
    va = np.zeros(int(cap[0]), np.float64)
    nnz = lib().orc_model_generator(model, _p(th), _p(dims_a), int(leaky), _p(rp), _p(ci), _p(va))
    if nnz < 0:
        raise ValueError("generator failed")
    return CSR(rp, ci[:nnz].copy(), va[:nnz].copy())


def poisson_logpmf(k: int, W: float) -> float:
    return float(lib().orc_poisson_logpmf(int(k), float(W)))


def pick_K(W: float, k_rule: int = K_TOL, eps_right: float = 1e-13):
    tail = np.zeros(1)
    K = int(lib().orc_pick_K(float(W), int(k_rule), float(eps_right), _p(tail)))
    return K, float(tail[0])


def weights(W: float, K: int):
    w = np.zeros(K + 1)
    total = float(lib().orc_weights(float(W), int(K), _p(w)))
    return w, total


def expv(A: CSR, rho0, t: float, omega_factor: float = 1.1, k_rule: int = K_TOL,
         eps_right: float = 1e-13, lump: bool = True):
    """Algorithm 2 in FP64; returns (rho(t), info dict)."""
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    assert rho0.shape == (A.n,)
    out = np.zeros(A.n)
    info = _Info()
    rc = lib().orc_expv(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(rho0), float(t),
                        float(omega_factor), int(k_rule), float(eps_right), int(lump), _p(out),
                        ctypes.cast(ctypes.byref(info), ctypes.c_void_p))
    if rc != 0:
        raise ValueError("oracle expv: bad input")
    return out, dict(omega=info.omega, W=info.W, eps_right=info.eps_right, residual=info.residual,
                     mass_in=info.mass_in, mass_out=info.mass_out, K=int(info.K))


def expv_times(A: CSR, rho0, times, **kw) -> np.ndarray:
    """Independent solves, one per time (the GPU path shares one sweep)."""
    return np.stack([expv(A, rho0, t, **kw)[0] for t in times])


def jump(A: CSR, x, omega_factor: float = 1.1) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(A.n)
    if lib().orc_jump(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), float(omega_factor), _p(x), _p(y)) != 0:
        raise ValueError("oracle jump: bad input")
    return y


def loglik(A: CSR, rho0, T, obs, omega_factor: float = 1.1, k_rule: int = K_TOL,
           eps_right: float = 1e-13) -> float:
    """sum_i c_i log rho(T_{j_i})_{s_i}; obs is an (I, 3) int array of
    (time index, state index, count)."""
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    obs = np.ascontiguousarray(obs, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(1)
    rc = lib().orc_loglik(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(rho0), len(T), _p(T),
                          obs.shape[0], _p(obs), float(omega_factor), int(k_rule), float(eps_right),
                          _p(out))
    if rc != 0:
        raise ValueError("oracle loglik: bad input")
    return float(out[0])


def loglik_marginal(A: CSR, rho0, T, groups, **kw) -> float:
    """Snapshot log-likelihood when part of the state is not observed (the
    gene state of the two-state and autoregulatory models, Secs. 3.1.2-3.1.3):
    sum_i c_i log sum_{s in S_i} rho(T_{j_i})_s.  groups is a list of
    (time index, list of state indices, count); independent solves per time."""
    rho = expv_times(A, rho0, T, **kw)
    total = 0.0
    for j, states, c in groups:
        p = float(np.sum(rho[int(j), np.asarray(states, dtype=np.int64)]))
        if not p > 0.0:
            return -np.inf
        total += c * np.log(p)
    return total
