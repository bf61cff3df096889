"""Thin ctypes binding of libmjp (include/mjp.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  Device
buffers are passed as torch CUDA tensors (their data pointers); the current
torch stream is used unless a stream is given.  Nothing in this module
computes any part of the method: if libmjp.so is missing or fails to load,
every call raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmjp.so")

MJP_OK, MJP_E_INVALID_ARG, MJP_E_NOT_GENERATOR, MJP_E_K_LIMIT, MJP_E_WORKSPACE, MJP_E_DEVICE, \
    MJP_E_NUMERIC, MJP_E_UNSUPPORTED = range(8)
STATUS_NAMES = ["MJP_OK", "MJP_E_INVALID_ARG", "MJP_E_NOT_GENERATOR", "MJP_E_K_LIMIT", "MJP_E_WORKSPACE",
                "MJP_E_DEVICE", "MJP_E_NUMERIC", "MJP_E_UNSUPPORTED"]
MJP_K_TOL, MJP_K_PAPER = 0, 1
MJP_CONSERVATIVE, MJP_LEAKY = 0, 1
MJP_VARIANT_AUTO, MJP_VARIANT_STEPWISE, MJP_VARIANT_PERSISTENT, MJP_VARIANT_PERSISTENT_FENCED = 0, 1, 2, 3
MJP_VARIANT_PERSISTENT_ONEJUMP = 4
MJP_VARIANT_PERSISTENT_TWOJUMP = 5
MJP_PATH_STEPWISE, MJP_PATH_PERSISTENT, MJP_PATH_PERSISTENT_FENCED, MJP_PATH_PERSISTENT_TWOJUMP = 1, 2, 3, 4
MJP_PATH_BATCHED_ITEM = 5
MJP_PATH_PERSISTENT_MULTIJUMP = 6
MJP_KRYLOV_AUTO, MJP_KRYLOV_PASSES, MJP_KRYLOV_FUSED = 0, 1, 2
MJP_MODEL_BD, MJP_MODEL_CASCADE2, MJP_MODEL_TWOSTATE, MJP_MODEL_AUTOREG = 0, 1, 2, 3
MJP_FLAG_NAN, MJP_FLAG_NEG, MJP_FLAG_UNDERFLOW_OBS, MJP_FLAG_OUT_OF_GRID, MJP_FLAG_K_LIMIT = 1, 2, 4, 8, 16
MJP_FLAG_SUBNORMAL_OBS = 32
MJP_LL_CLASSES, MJP_LL_MAX_SHAPES = 4, 16


class MjpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 8 else status}: {msg}")


class mjp_opts(ctypes.Structure):
    _fields_ = [("omega_factor", ctypes.c_double), ("tol", ctypes.c_double), ("k_rule", ctypes.c_int32),
                ("truncation", ctypes.c_int32), ("renorm_every", ctypes.c_int32), ("lump", ctypes.c_int32),
                ("k_cap", ctypes.c_int64), ("variant", ctypes.c_int32), ("barrier_timeout_us", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 6)]


class mjp_info(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("W", ctypes.c_double), ("eps_left", ctypes.c_double),
                ("eps_right", ctypes.c_double), ("residual", ctypes.c_double), ("mass_in", ctypes.c_double),
                ("mass_out", ctypes.c_double), ("K", ctypes.c_int32), ("L", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("path", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class mjp_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class mjp_model(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("dims", ctypes.c_int32 * 2), ("theta", ctypes.c_double * 8)]


class mjp_obs(ctypes.Structure):
    _fields_ = [("n_t", ctypes.c_int32), ("T_h", ctypes.c_void_p), ("n_obs", ctypes.c_int32),
                ("obs_h", ctypes.c_void_p), ("x0", ctypes.c_int32 * 2)]


class mjp_sampler_cfg(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("dims", ctypes.c_int32 * 2), ("chains", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("prior_mu", ctypes.c_double), ("prior_sigma", ctypes.c_double)]


class mjp_mlp_cfg(ctypes.Structure):
    _fields_ = [("in_dim", ctypes.c_int32), ("width", ctypes.c_int32), ("depth", ctypes.c_int32)]


class mjp_train_cfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps_adam", ctypes.c_float),
                ("weight_decay", ctypes.c_float), ("seed", ctypes.c_uint64)]


class mjp_krylov_opts(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_int32), ("variant", ctypes.c_int32), ("dt_factor", ctypes.c_double),
                ("reserved", ctypes.c_int32 * 6)]


class mjp_krylov_info(ctypes.Structure):
    _fields_ = [("m_theta", ctypes.c_double), ("dt", ctypes.c_double), ("steps", ctypes.c_int64),
                ("kappa", ctypes.c_int32), ("fused", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class mjp_ll_shape(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("cells", ctypes.c_int32), ("max_states", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


class mjp_ll_tune_report(ctypes.Structure):
    _fields_ = [("items", ctypes.c_int32 * MJP_LL_CLASSES), ("chosen", ctypes.c_int32 * MJP_LL_CLASSES),
                ("ms", (ctypes.c_float * MJP_LL_MAX_SHAPES) * MJP_LL_CLASSES)]


class mjp_rk4_opts(ctypes.Structure):
    _fields_ = [("dt_factor", ctypes.c_double), ("reserved", ctypes.c_int32 * 6)]


class mjp_rk4_info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_double), ("dt", ctypes.c_double), ("steps", ctypes.c_int64),
                ("reserved", ctypes.c_int32 * 6)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


_lib = None

# (name, restype, argtypes) of every exported function
_P = ctypes.c_void_p
_SIGS = [
    ("mjp_opts_default", None, [_P]),
    ("mjp_model_csr_size", ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    ("mjp_model_csr", ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    ("mjp_plan_create_csr", ctypes.c_int, [_P, _P, _P]),
    ("mjp_plan_create_stencil", ctypes.c_int, [_P, _P, _P]),
    ("mjp_plan_destroy", None, [_P]),
    ("mjp_plan_n", ctypes.c_int32, [_P]),
    ("mjp_expv", ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P, _P]),
    ("mjp_expv_batched", ctypes.c_int, [ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P]),
    ("mjp_probe_exchange", ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    ("mjp_probe_exchange2", ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    ("mjp_loglik", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P]),
    ("mjp_loglik_set_kernel", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32]),
    ("mjp_loglik_cluster_config", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("mjp_loglik_noalloc", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P]),
    ("mjp_loglik_noalloc_bytes", ctypes.c_int64, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    ("mjp_loglik_noalloc_capacity", ctypes.c_int64, []),
    ("mjp_loglik_max_states", ctypes.c_int32, []),
    ("mjp_loglik_num_shapes", ctypes.c_int32, []),
    ("mjp_loglik_shape", ctypes.c_int, [ctypes.c_int32, _P]),
    ("mjp_loglik_class_limit", ctypes.c_int32, [ctypes.c_int32]),
    ("mjp_loglik_set_shapes", ctypes.c_int, [ctypes.c_int32, _P]),
    ("mjp_loglik_get_shapes", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _P]),
    ("mjp_loglik_save_shapes", ctypes.c_int, [ctypes.c_char_p]),
    ("mjp_loglik_load_shapes", ctypes.c_int, [ctypes.c_char_p]),
    ("mjp_loglik_tune", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P, _P, ctypes.c_int32, _P,
                                       _P]),
    ("mjp_jump_probs", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, _P]),
    ("mjp_surrogate_create", ctypes.c_int, [_P, ctypes.c_uint64, _P]),
    ("mjp_surrogate_destroy", None, [_P]),
    ("mjp_surrogate_train", ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, _P]),
    ("mjp_surrogate_infer", ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P]),
    ("mjp_surrogate_grad", ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, _P]),
    ("mjp_surrogate_num_params", ctypes.c_int64, [_P]),
    ("mjp_surrogate_get_params", ctypes.c_int, [_P, _P, ctypes.c_int64]),
    ("mjp_surrogate_set_params", ctypes.c_int, [_P, _P, ctypes.c_int64]),
    ("mjp_surrogate_save", ctypes.c_int, [_P, ctypes.c_char_p]),
    ("mjp_surrogate_load", ctypes.c_int, [ctypes.c_char_p, _P]),
    ("mjp_krylov_opts_default", None, [_P]),
    ("mjp_krylov_create", ctypes.c_int, [_P, _P, _P]),
    ("mjp_krylov_destroy", None, [_P]),
    ("mjp_krylov_n", ctypes.c_int32, [_P]),
    ("mjp_krylov_expv", ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P, _P]),
    ("mjp_rk4_opts_default", None, [_P]),
    ("mjp_rk4_create", ctypes.c_int, [ctypes.c_int32, _P, _P, _P]),
    ("mjp_rk4_create_stencil", ctypes.c_int, [_P, _P, _P]),
    ("mjp_rk4_destroy", None, [_P]),
    ("mjp_rk4_n", ctypes.c_int32, [_P]),
    ("mjp_rk4_set_schedule", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    ("mjp_rk4_expv", ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P, _P]),
    ("mjp_last_error", ctypes.c_char_p, []),
    ("mjp_version", ctypes.c_char_p, []),
    ("mjp_shutdown", ctypes.c_int, []),
    ("mjp_sampler_cfg_default", None, [_P]),
    ("mjp_sampler_create", ctypes.c_int, [_P, _P, _P, _P]),
    ("mjp_sampler_destroy", None, [_P]),
    ("mjp_sampler_set_proposal", ctypes.c_int, [_P, _P]),
    ("mjp_sampler_set_screen", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_double, ctypes.c_double]),
    ("mjp_sampler_init", ctypes.c_int, [_P, _P, _P]),
    ("mjp_sampler_run", ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, _P]),
    ("mjp_sampler_get_state", ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    ("mjp_sampler_set_state", ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    ("mjp_philox4x32_10", None, [_P, _P, _P]),
    ("mjp_poisson_fill", ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint32, _P, ctypes.c_int32, _P, _P]),
    ("mjp_jmjp_create", ctypes.c_int, [_P, _P, _P, _P]),
    ("mjp_jmjp_destroy", None, [_P]),
    ("mjp_jmjp_set_proposal", ctypes.c_int, [_P, _P]),
    ("mjp_jmjp_init", ctypes.c_int, [_P, _P, ctypes.c_int32, _P]),
    ("mjp_jmjp_run", ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, _P]),
    ("mjp_jmjp_counters", ctypes.c_int, [_P, _P, _P]),
    ("mjp_philox_fill", ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                       ctypes.c_int32, _P, _P]),
]


def _shutdown_at_exit():
    # free the library's own device tables while the HIP runtime is still up
    if _lib is not None:
        _lib.mjp_shutdown()


def lib():
    """Load libmjp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2312_05647_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        atexit.register(_shutdown_at_exit)
    return _lib


def mjp_shutdown() -> None:
    _check(lib().mjp_shutdown())


def _check(status: int):
    if status != MJP_OK:
        raise MjpError(status, lib().mjp_last_error().decode())


def _ptr(x) -> int:
    """Data pointer of a torch tensor or numpy array (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


# ---------------------------------------------------------------- options

def mjp_opts_default(**over) -> mjp_opts:
    o = mjp_opts()
    lib().mjp_opts_default(ctypes.byref(o))
    for k, v in over.items():
        setattr(o, k, v)
    return o


def make_model(model: int, theta, dims) -> mjp_model:
    m = mjp_model()
    m.model = model
    d = list(dims) + [1] * (2 - len(dims))
    m.dims[0], m.dims[1] = int(d[0]), int(d[1])
    for i, v in enumerate(theta):
        m.theta[i] = float(v)
    return m


def mjp_model_csr(model: mjp_model, truncation: int = MJP_CONSERVATIVE):
    """Host CSR (row_ptr int32, col int32, val float64) of a built-in model."""
    n = ctypes.c_int32()
    nnz = ctypes.c_int32()
    _check(lib().mjp_model_csr_size(ctypes.byref(model), truncation, ctypes.byref(n), ctypes.byref(nnz)))
    rp = np.zeros(n.value + 1, np.int32)
    ci = np.zeros(nnz.value, np.int32)
    va = np.zeros(nnz.value, np.float64)
    _check(lib().mjp_model_csr(ctypes.byref(model), truncation, _ptr(rp), _ptr(ci), _ptr(va)))
    return rp, ci, va


# ---------------------------------------------------------------- plans

def mjp_plan_create_csr(row_ptr, col, val, opts: mjp_opts | None = None) -> int:
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    A = mjp_csr(len(row_ptr) - 1, len(col), _ptr(row_ptr), _ptr(col), _ptr(val))
    opts = opts or mjp_opts_default()
    h = ctypes.c_void_p()
    _check(lib().mjp_plan_create_csr(ctypes.byref(A), ctypes.byref(opts), ctypes.byref(h)))
    return h.value


def mjp_plan_create_stencil(model: mjp_model, opts: mjp_opts | None = None) -> int:
    opts = opts or mjp_opts_default()
    h = ctypes.c_void_p()
    _check(lib().mjp_plan_create_stencil(ctypes.byref(model), ctypes.byref(opts), ctypes.byref(h)))
    return h.value


def mjp_plan_destroy(plan: int) -> None:
    lib().mjp_plan_destroy(plan)


def mjp_plan_n(plan: int) -> int:
    return int(lib().mjp_plan_n(plan))


# -------------------------------------------------------------- solvers

def mjp_expv(plan: int, rho0, times, out, info: bool = False, stream=None):
    """out[j] = rho(times[j]); rho0 [N] and out [n_t, N] are float32 CUDA
    tensors.  Returns a list of info dicts when info=True (synchronous)."""
    t = np.ascontiguousarray(times, dtype=np.float64).reshape(-1)
    inf = (mjp_info * len(t))() if info else None
    _check(lib().mjp_expv(plan, _ptr(rho0), len(t), _ptr(t), _ptr(out),
                          ctypes.cast(inf, ctypes.c_void_p) if info else None, _stream(stream)))
    return [i.as_dict() for i in inf] if info else None


def mjp_probe_exchange(plan: int, rounds: int, stream=None) -> float:
    """Microseconds per round of the two-jump sweep's communication alone on
    this plan's launch configuration (a measurement aid)."""
    us = ctypes.c_double()
    _check(lib().mjp_probe_exchange(plan, rounds, ctypes.byref(us), _stream(stream)))
    return us.value


def mjp_probe_exchange2(plan, rounds: int, stream=None):
    """(microseconds per round, jumps per round) of the plan's sweep's exchange floor."""
    us = ctypes.c_double()
    j = ctypes.c_int32()
    _check(lib().mjp_probe_exchange2(plan, rounds, ctypes.byref(us), ctypes.byref(j), _stream(stream)))
    return us.value, j.value


def _row_ptrs(x, B):
    """Per-item device pointers: a list of tensors, or one contiguous tensor
    whose leading dimension is the item (rows of [B, ...])."""
    if hasattr(x, "data_ptr") and hasattr(x, "is_contiguous"):
        assert x.is_contiguous() and x.shape[0] == B, "a batched tensor must be contiguous with B rows"
        base, step = x.data_ptr(), x[0].numel() * x.element_size()
        return [base + b * step for b in range(B)]
    return [_ptr(r) for r in x]


def mjp_expv_batched(plans, rho0s, times_list, outs, info: bool = False, stream=None):
    """rho0s: list of [N_b] tensors or one contiguous [B, N] tensor; outs:
    list of [n_t_b, N_b] tensors or one contiguous [B, n_t, N] tensor."""
    B = len(plans)
    P = (ctypes.c_void_p * B)(*plans)
    R = (ctypes.c_void_p * B)(*_row_ptrs(rho0s, B))
    O = (ctypes.c_void_p * B)(*_row_ptrs(outs, B))
    conv = {}  # (array, length, pointer) per distinct times object: a batch often repeats one list
    keep, nts, tps = [], [], []
    for t in times_list:
        c = conv.get(id(t))
        if c is None:
            a = np.ascontiguousarray(t, dtype=np.float64).reshape(-1)
            keep.append(a)
            c = conv[id(t)] = (len(a), a.ctypes.data)
        nts.append(c[0])
        tps.append(c[1])
    NT = (ctypes.c_int32 * B)(*nts)
    TP = (ctypes.c_void_p * B)(*tps)
    total = sum(nts)
    inf = (mjp_info * total)() if info else None
    _check(lib().mjp_expv_batched(B, P, R, NT, TP, O, ctypes.cast(inf, ctypes.c_void_p) if info else None,
                                  _stream(stream)))
    return [i.as_dict() for i in inf] if info else None


# ------------------------------------------------------- Krylov (Method #5)

def mjp_krylov_opts_default(**kw) -> mjp_krylov_opts:
    o = mjp_krylov_opts()
    lib().mjp_krylov_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def mjp_krylov_create(row_ptr, col, val, opts: mjp_krylov_opts | None = None) -> int:
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    A = mjp_csr(len(row_ptr) - 1, len(col), _ptr(row_ptr), _ptr(col), _ptr(val))
    opts = opts or mjp_krylov_opts_default()
    h = ctypes.c_void_p()
    _check(lib().mjp_krylov_create(ctypes.byref(A), ctypes.byref(opts), ctypes.byref(h)))
    return h.value


def mjp_krylov_destroy(k: int) -> None:
    lib().mjp_krylov_destroy(k)


def mjp_krylov_n(k: int) -> int:
    return int(lib().mjp_krylov_n(k))


def mjp_krylov_expv(k: int, rho0, times, out, stream=None) -> dict:
    """out[j] = rho(times[j]); rho0 [N] and out [n_t, N] are float64 CUDA
    tensors.  Returns the info dict (step count) filled on the host."""
    t = np.ascontiguousarray(times, dtype=np.float64).reshape(-1)
    inf = mjp_krylov_info()
    _check(lib().mjp_krylov_expv(k, _ptr(rho0), len(t), _ptr(t), _ptr(out), ctypes.byref(inf), _stream(stream)))
    return inf.as_dict()


# -------------------------------------------------- Runge-Kutta (Method #4)

def mjp_rk4_opts_default(**kw) -> mjp_rk4_opts:
    o = mjp_rk4_opts()
    lib().mjp_rk4_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def mjp_rk4_create(channels, opts: mjp_rk4_opts | None = None) -> int:
    """channels: list of host CSR triples (row_ptr, col, val), one per A_c."""
    keep = [(np.ascontiguousarray(rp, dtype=np.int32), np.ascontiguousarray(ci, dtype=np.int32),
             np.ascontiguousarray(va, dtype=np.float64)) for rp, ci, va in channels]
    arr = (mjp_csr * len(keep))(*[mjp_csr(len(rp) - 1, len(ci), _ptr(rp), _ptr(ci), _ptr(va))
                                   for rp, ci, va in keep])
    opts = opts or mjp_rk4_opts_default()
    h = ctypes.c_void_p()
    _check(lib().mjp_rk4_create(len(keep), arr, ctypes.byref(opts), ctypes.byref(h)))
    return h.value


def mjp_rk4_create_stencil(model: mjp_model, opts: mjp_rk4_opts | None = None) -> int:
    """Birth-death or cascade model given by its rates; channels = its reactions."""
    opts = opts or mjp_rk4_opts_default()
    h = ctypes.c_void_p()
    _check(lib().mjp_rk4_create_stencil(ctypes.byref(model), ctypes.byref(opts), ctypes.byref(h)))
    return h.value


def mjp_rk4_set_schedule(k: int, channel: int, t_knots, g_knots) -> None:
    t = np.ascontiguousarray(t_knots, dtype=np.float64).reshape(-1)
    g = np.ascontiguousarray(g_knots, dtype=np.float64).reshape(-1)
    if len(t) != len(g):
        raise ValueError("t_knots and g_knots differ in length")
    _check(lib().mjp_rk4_set_schedule(k, channel, len(t), _ptr(t), _ptr(g)))


def mjp_rk4_destroy(k: int) -> None:
    lib().mjp_rk4_destroy(k)


def mjp_rk4_n(k: int) -> int:
    return int(lib().mjp_rk4_n(k))


def mjp_rk4_expv(k: int, rho0, times, out, stream=None) -> dict:
    """out[j] = rho(times[j]); rho0 [N] and out [n_t, N] are float64 CUDA
    tensors.  Returns the info dict (m, dt, steps) filled on the host."""
    t = np.ascontiguousarray(times, dtype=np.float64).reshape(-1)
    inf = mjp_rk4_info()
    _check(lib().mjp_rk4_expv(k, _ptr(rho0), len(t), _ptr(t), _ptr(out), ctypes.byref(inf), _stream(stream)))
    return inf.as_dict()


def make_obs(T, obs, x0=(0, 0)):
    """Keeps the host arrays alive alongside the struct."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    obs = np.ascontiguousarray(obs, dtype=np.int32).reshape(-1, 4)
    o = mjp_obs(len(T), _ptr(T), obs.shape[0], _ptr(obs), (ctypes.c_int32 * 2)(*x0))
    o._keep = (T, obs)
    return o


def mjp_loglik(model: int, theta, dims, obs: mjp_obs, out, opts: mjp_opts | None = None, info=None,
               stream=None) -> None:
    """theta [B, 4] float64, dims [B, 2] int32, out [B] float64: CUDA tensors;
    info: optional CUDA uint8 tensor of B * sizeof(mjp_info) bytes."""
    opts = opts or mjp_opts_default()
    B = int(out.shape[0])
    _check(lib().mjp_loglik(model, B, _ptr(theta), _ptr(dims), ctypes.byref(obs), ctypes.byref(opts), _ptr(out),
                            _ptr(info), _stream(stream)))


MJP_LL_KERNEL_AUTO, MJP_LL_KERNEL_CELLS = 0, 1


def mjp_loglik_cluster_config() -> dict:
    v = [ctypes.c_int32() for _ in range(5)]
    _check(lib().mjp_loglik_cluster_config(*[ctypes.byref(x) for x in v]))
    return dict(zip(("clusters", "per_cu", "cooperative", "group", "max_states"), (x.value for x in v)))


def mjp_loglik_set_kernel(model: int, kernel: int) -> None:
    _check(lib().mjp_loglik_set_kernel(model, kernel))


def mjp_loglik_noalloc(model: int, theta, dims, obs: mjp_obs, out, opts: mjp_opts | None = None, info=None,
                       stream=None) -> None:
    """mjp_loglik with the call's tables in the library's fixed device array
    (no allocation); same arguments."""
    opts = opts or mjp_opts_default()
    B = int(out.shape[0])
    _check(lib().mjp_loglik_noalloc(model, B, _ptr(theta), _ptr(dims), ctypes.byref(obs), ctypes.byref(opts),
                                    _ptr(out), _ptr(info), _stream(stream)))


def mjp_loglik_noalloc_bytes(B: int, n_t: int, n_obs: int) -> int:
    return int(lib().mjp_loglik_noalloc_bytes(B, n_t, n_obs))


def mjp_loglik_noalloc_capacity() -> int:
    return int(lib().mjp_loglik_noalloc_capacity())


def mjp_jump_probs(model: int, theta, dims, obs: mjp_obs, k, logphi, omega=None, opts: mjp_opts | None = None,
                   stream=None) -> None:
    """J-MJP state probabilities: logphi[b, i] = log p(s_i | k[b, i], theta[b]).
    theta [B, P] float64, dims [B, 2] int32, k [B, I] int32, logphi [B, I]
    float64, omega [B] float64 or None: CUDA tensors; obs records of count 1."""
    opts = opts or mjp_opts_default()
    B = int(logphi.shape[0])
    _check(lib().mjp_jump_probs(model, B, _ptr(theta), _ptr(dims), ctypes.byref(obs), _ptr(k), ctypes.byref(opts),
                                _ptr(logphi), _ptr(omega), _stream(stream)))


def mjp_loglik_max_states() -> int:
    return int(lib().mjp_loglik_max_states())


def mjp_loglik_shapes() -> list:
    """The launch-shape table: one dict per shape id."""
    out = []
    for i in range(int(lib().mjp_loglik_num_shapes())):
        sh = mjp_ll_shape()
        _check(lib().mjp_loglik_shape(i, ctypes.byref(sh)))
        out.append({"threads": sh.threads, "cells": sh.cells, "max_states": sh.max_states,
                    "lds_bytes": sh.lds_bytes})
    return out


def mjp_loglik_class_limits() -> list:
    return [int(lib().mjp_loglik_class_limit(c)) for c in range(MJP_LL_CLASSES)]


def mjp_loglik_set_shapes(model: int, ids) -> None:
    """Shape id per size class for `model` on the current device (-1 = default)."""
    a = (ctypes.c_int32 * MJP_LL_CLASSES)(*[int(i) for i in ids])
    _check(lib().mjp_loglik_set_shapes(model, a))


def mjp_loglik_get_shapes(model: int, n_rec: int = 0) -> list:
    a = (ctypes.c_int32 * MJP_LL_CLASSES)()
    _check(lib().mjp_loglik_get_shapes(model, n_rec, a))
    return list(a)


def mjp_loglik_save_shapes(path: str) -> None:
    _check(lib().mjp_loglik_save_shapes(os.fsencode(path)))


def mjp_loglik_load_shapes(path: str) -> None:
    _check(lib().mjp_loglik_load_shapes(os.fsencode(path)))


def mjp_loglik_tune(model: int, theta, dims, obs: mjp_obs, out, opts: mjp_opts | None = None, info=None,
                    reps: int = 2, stream=None) -> dict:
    """Times every eligible shape per size class on this batch, keeps the
    fastest; `out` (and `info`) then hold the batch's log-likelihoods."""
    opts = opts or mjp_opts_default()
    B = int(out.shape[0])
    rep = mjp_ll_tune_report()
    _check(lib().mjp_loglik_tune(model, B, _ptr(theta), _ptr(dims), ctypes.byref(obs), ctypes.byref(opts), _ptr(out),
                                 _ptr(info), reps, ctypes.byref(rep), _stream(stream)))
    return {"items": list(rep.items), "chosen": list(rep.chosen),
            "ms": [[float(v) for v in row] for row in rep.ms]}


# ------------------------------------------------------------ surrogate

def mjp_surrogate_create(in_dim=4, width=256, depth=3, seed=0) -> int:
    cfg = mjp_mlp_cfg(in_dim, width, depth)
    h = ctypes.c_void_p()
    _check(lib().mjp_surrogate_create(ctypes.byref(cfg), seed, ctypes.byref(h)))
    return h.value


def mjp_surrogate_destroy(s: int) -> None:
    lib().mjp_surrogate_destroy(s)


def mjp_surrogate_train(s: int, x, y, cfg: mjp_train_cfg, losses: bool = True, stream=None):
    n = int(y.shape[0])
    buf = np.zeros(cfg.epochs, np.float32) if losses else None
    _check(lib().mjp_surrogate_train(s, _ptr(x), _ptr(y), n, ctypes.byref(cfg), _ptr(buf), _stream(stream)))
    return buf


def mjp_surrogate_infer(s: int, x, y, stream=None) -> None:
    _check(lib().mjp_surrogate_infer(s, _ptr(x), int(x.shape[0]), _ptr(y), _stream(stream)))


def mjp_surrogate_grad(s: int, x, y, stream=None):
    """(loss, gradient as float32 numpy) of the MSE on one batch."""
    g = np.zeros(mjp_surrogate_num_params(s), np.float32)
    loss = np.zeros(1, np.float32)
    _check(lib().mjp_surrogate_grad(s, _ptr(x), _ptr(y), int(y.shape[0]), _ptr(g), _ptr(loss), _stream(stream)))
    return float(loss[0]), g


def mjp_train_cfg_default(**over) -> mjp_train_cfg:
    c = mjp_train_cfg(epochs=10, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999, eps_adam=1e-8, weight_decay=0.0, seed=0)
    for k, v in over.items():
        setattr(c, k, v)
    return c


def mjp_surrogate_num_params(s: int) -> int:
    return int(lib().mjp_surrogate_num_params(s))


def mjp_surrogate_get_params(s: int) -> np.ndarray:
    buf = np.zeros(mjp_surrogate_num_params(s), np.float32)
    _check(lib().mjp_surrogate_get_params(s, _ptr(buf), buf.size))
    return buf


def mjp_surrogate_set_params(s: int, params) -> None:
    buf = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().mjp_surrogate_set_params(s, _ptr(buf), buf.size))


def mjp_surrogate_save(s: int, path: str) -> None:
    _check(lib().mjp_surrogate_save(s, path.encode()))


def mjp_surrogate_load(path: str) -> int:
    h = ctypes.c_void_p()
    _check(lib().mjp_surrogate_load(path.encode(), ctypes.byref(h)))
    return h.value


def mjp_last_error() -> str:
    return lib().mjp_last_error().decode()


def mjp_version() -> str:
    return lib().mjp_version().decode()


# ------------------------------------------------------- device samplers

def mjp_sampler_cfg_default(**kw) -> mjp_sampler_cfg:
    c = mjp_sampler_cfg()
    lib().mjp_sampler_cfg_default(ctypes.byref(c))
    for k, v in kw.items():
        if k == "dims":
            c.dims = (ctypes.c_int32 * 2)(*v)
        else:
            setattr(c, k, v)
    return c


def mjp_sampler_create(cfg: mjp_sampler_cfg, obs: mjp_obs, opts: mjp_opts | None = None) -> int:
    h = ctypes.c_void_p()
    _check(lib().mjp_sampler_create(ctypes.byref(cfg), ctypes.byref(obs), ctypes.byref(opts or mjp_opts_default()),
                                    ctypes.byref(h)))
    return h.value


def mjp_sampler_destroy(h) -> None:
    lib().mjp_sampler_destroy(h)


def mjp_sampler_set_proposal(h, chol) -> None:
    L = np.ascontiguousarray(chol, dtype=np.float64)
    _check(lib().mjp_sampler_set_proposal(h, _ptr(L)))


def mjp_sampler_set_screen(h, screen, psi_mean=None, psi_std=None, ll_mean=0.0, ll_std=1.0) -> None:
    if screen is None:
        _check(lib().mjp_sampler_set_screen(h, None, None, None, 0.0, 1.0))
        return
    m = np.ascontiguousarray(psi_mean, dtype=np.float64)
    sd = np.ascontiguousarray(psi_std, dtype=np.float64)
    _check(lib().mjp_sampler_set_screen(h, screen, _ptr(m), _ptr(sd), float(ll_mean), float(ll_std)))


def mjp_sampler_init(h, psi0, stream=None) -> None:
    _check(lib().mjp_sampler_init(h, _ptr(psi0), _stream(stream)))


def mjp_sampler_run(h, steps: int, samples=None, stream=None) -> None:
    """samples: None or a device float64 tensor [ring, C, d]."""
    ring = int(samples.shape[0]) if samples is not None else 0
    _check(lib().mjp_sampler_run(h, int(steps), _ptr(samples), ring, _stream(stream)))


def mjp_sampler_get_state(h, C: int, d: int, stream=None):
    psi = np.empty((C, d)); lp = np.empty(C); sc = np.empty(C); ctr = np.zeros(4, np.uint64)
    _check(lib().mjp_sampler_get_state(h, _ptr(psi), _ptr(lp), _ptr(sc), _ptr(ctr), _stream(stream)))
    return {"psi": psi, "lp": lp, "sc": sc, "counters": ctr}


def mjp_sampler_set_state(h, state, stream=None) -> None:
    psi = np.ascontiguousarray(state["psi"], dtype=np.float64)
    lp = np.ascontiguousarray(state["lp"], dtype=np.float64)
    sc = np.ascontiguousarray(state["sc"], dtype=np.float64)
    ctr = np.ascontiguousarray(state["counters"], dtype=np.uint64)
    _check(lib().mjp_sampler_set_state(h, _ptr(psi), _ptr(lp), _ptr(sc), _ptr(ctr), _stream(stream)))


def mjp_philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().mjp_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def mjp_philox_fill(key: int, c1: int, c2: int, c3: int, out, stream=None) -> None:
    """out: device uint32-sized tensor of 4 n words (torch int32 works)."""
    n = out.numel() // 4
    _check(lib().mjp_philox_fill(int(key), c1, c2, c3, n, _ptr(out), _stream(stream)))


def mjp_poisson_fill(key: int, c1: int, lam, out, stream=None) -> None:
    """lam: device float64 tensor [n]; out: device int32 tensor [n]."""
    _check(lib().mjp_poisson_fill(int(key), int(c1), _ptr(lam), int(lam.numel()), _ptr(out), _stream(stream)))


def mjp_jmjp_create(cfg: mjp_sampler_cfg, obs: mjp_obs, opts: mjp_opts | None = None) -> int:
    h = ctypes.c_void_p()
    _check(lib().mjp_jmjp_create(ctypes.byref(cfg), ctypes.byref(obs), ctypes.byref(opts or mjp_opts_default()),
                                 ctypes.byref(h)))
    return h.value


def mjp_jmjp_destroy(h) -> None:
    lib().mjp_jmjp_destroy(h)


def mjp_jmjp_set_proposal(h, chol) -> None:
    L = np.ascontiguousarray(chol, dtype=np.float64)
    _check(lib().mjp_jmjp_set_proposal(h, _ptr(L)))


def mjp_jmjp_init(h, psi0, k_burn: int = 20, stream=None) -> None:
    _check(lib().mjp_jmjp_init(h, _ptr(psi0), int(k_burn), _stream(stream)))


def mjp_jmjp_run(h, steps: int, samples=None, stream=None) -> None:
    ring = int(samples.shape[0]) if samples is not None else 0
    _check(lib().mjp_jmjp_run(h, int(steps), _ptr(samples), ring, _stream(stream)))


def mjp_jmjp_counters(h, stream=None) -> np.ndarray:
    ctr = np.zeros(4, np.uint64)
    _check(lib().mjp_jmjp_counters(h, _ptr(ctr), _stream(stream)))
    return ctr
