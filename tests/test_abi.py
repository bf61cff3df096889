"""C-ABI checks that need no GPU: the library loads, exports every function
include/mjp.h declares, builds model generators identical to the oracle's
independent ones, and rejects invalid calls on the host before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2312_05647_amd import mjp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mjp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(mjp_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    L = mjp.lib()
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    bound = {n for n, _, _ in mjp._SIGS}
    assert set(names) == bound, set(names) ^ bound


def test_shutdown_without_device_work_is_a_no_op():
    # nothing was allocated by the library: no device call is made
    assert mjp.lib().mjp_shutdown() == mjp.MJP_OK
    assert mjp.lib().mjp_shutdown() == mjp.MJP_OK


def test_version_and_defaults():
    assert "gfx950" in mjp.mjp_version()
    o = mjp.mjp_opts_default()
    assert o.omega_factor == 1.1 and o.tol == 1e-9 and o.lump == 1
    assert o.k_rule == mjp.MJP_K_TOL and o.truncation == mjp.MJP_CONSERVATIVE


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes struct of the binding has the size and field offsets the
    C compiler gives the header's struct."""
    import subprocess
    structs = {"mjp_opts": mjp.mjp_opts, "mjp_info": mjp.mjp_info, "mjp_csr": mjp.mjp_csr,
               "mjp_model": mjp.mjp_model, "mjp_obs": mjp.mjp_obs, "mjp_mlp_cfg": mjp.mjp_mlp_cfg,
               "mjp_train_cfg": mjp.mjp_train_cfg, "mjp_krylov_opts": mjp.mjp_krylov_opts,
               "mjp_krylov_info": mjp.mjp_krylov_info,
               "mjp_rk4_opts": mjp.mjp_rk4_opts, "mjp_rk4_info": mjp.mjp_rk4_info,
               "mjp_ll_shape": mjp.mjp_ll_shape, "mjp_ll_tune_report": mjp.mjp_ll_tune_report,
               "mjp_sampler_cfg": mjp.mjp_sampler_cfg}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mjp.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)


@pytest.mark.parametrize("leaky", [0, 1])
@pytest.mark.parametrize("case", [(0, [500.0, 1.0], [1000]), (0, [3.0, 0.0], [9]), (1, [200.0, 1.0, 0.5, 0.5], [30, 20]),
                                  (1, [5.0, 0.7, 0.0, 2.0], [7, 5]), (1, [1.0, 2.0, 3.0, 4.0], [1, 6]),
                                  (2, [100.0, 1.0, 2.0, 1.0], [250]), (2, [3.0, 0.5, 0.0, 1.5], [1]),
                                  (3, [5.0, 0.25, 1.0, 0.1, 0.1, 0.05], [20, 40]),
                                  (3, [2.5, 0.4, 1.0, 0.3, 0.0, 0.05], [1, 3])])
def test_model_csr_matches_oracle(orc, case, leaky):
    model, theta, dims = case
    rp, ci, va = mjp.mjp_model_csr(mjp.make_model(model, theta, dims), leaky)
    ref = orc.model_generator(model, theta, dims, leaky=bool(leaky))
    assert np.array_equal(rp.astype(np.int64), ref.row_ptr)
    assert np.array_equal(ci, ref.col)
    assert np.allclose(va, ref.val, rtol=1e-14, atol=0)


def _csr(rp, ci, va):
    return (np.asarray(rp, np.int32), np.asarray(ci, np.int32), np.asarray(va, np.float64))


GOOD = _csr([0, 2, 4], [0, 1, 0, 1], [-1.0, 1.0, 2.0, -2.0])


def status_of(fn, *a, **k):
    try:
        fn(*a, **k)
    except mjp.MjpError as e:
        return e.status
    return mjp.MJP_OK


@pytest.mark.parametrize("bad,expect", [
    (_csr([0, 2, 4], [0, 1, 0, 1], [-1.0, -1.0, 2.0, -2.0]), mjp.MJP_E_NOT_GENERATOR),   # negative rate
    (_csr([0, 2, 4], [0, 1, 0, 1], [-1.5, 1.0, 2.0, -2.0]), mjp.MJP_E_NOT_GENERATOR),    # row sum != 0
    (_csr([0, 2, 4], [1, 0, 0, 1], [1.0, -1.0, 2.0, -2.0]), mjp.MJP_E_INVALID_ARG),      # unsorted
    (_csr([0, 2, 4], [0, 2, 0, 1], [-1.0, 1.0, 2.0, -2.0]), mjp.MJP_E_INVALID_ARG),      # column out of range
    (_csr([0, 3, 4], [0, 1, 0, 1], [-1.0, 1.0, 2.0, -2.0]), mjp.MJP_E_INVALID_ARG),      # row_ptr end != nnz
    (_csr([0, 2, 4], [0, 1, 0, 1], [-1.0, np.nan, 2.0, -2.0]), mjp.MJP_E_INVALID_ARG),   # non-finite
    (_csr([0], [], []), mjp.MJP_E_INVALID_ARG),                                          # n = 0
])
def test_csr_validation(bad, expect):
    assert status_of(mjp.mjp_plan_create_csr, *bad) == expect


def test_leaky_rows_may_lose_but_not_gain_mass():
    gain = _csr([0, 2, 4], [0, 1, 0, 1], [-0.5, 1.0, 2.0, -2.0])
    assert status_of(mjp.mjp_plan_create_csr, *gain, mjp.mjp_opts_default(truncation=mjp.MJP_LEAKY, renorm_every=0)) \
        == mjp.MJP_E_NOT_GENERATOR


@pytest.mark.parametrize("over", [dict(omega_factor=1.0), dict(omega_factor=float("nan")), dict(tol=0.0),
                                  dict(tol=1.0), dict(k_rule=5), dict(truncation=3), dict(renorm_every=-1),
                                  dict(truncation=1, renorm_every=8), dict(lump=2), dict(k_cap=0),
                                  dict(variant=9)])
def test_option_validation(over):
    o = mjp.mjp_opts_default(**over)
    assert status_of(mjp.mjp_plan_create_csr, *GOOD, o) == mjp.MJP_E_INVALID_ARG
    m = mjp.make_model(mjp.MJP_MODEL_BD, [1.0, 1.0], [5])
    assert status_of(mjp.mjp_plan_create_stencil, m, o) == mjp.MJP_E_INVALID_ARG


def test_reserved_option_fields_must_be_zero():
    o = mjp.mjp_opts_default()
    o.reserved[3] = 1
    assert status_of(mjp.mjp_plan_create_csr, *GOOD, o) == mjp.MJP_E_INVALID_ARG


@pytest.mark.parametrize("model,theta,dims", [(7, [1.0], [3]), (0, [-1.0, 1.0], [5]), (0, [1.0, 1.0], [0]),
                                              (0, [1.0, 1.0], [5, 2]), (1, [1.0, 1.0, np.inf, 1.0], [4, 4]),
                                              (1, [1.0] * 4, [0, 4])])
def test_model_validation(model, theta, dims):
    m = mjp.make_model(model, theta, dims)
    assert status_of(mjp.mjp_plan_create_stencil, m) == mjp.MJP_E_INVALID_ARG
    assert status_of(mjp.mjp_model_csr, m) == mjp.MJP_E_INVALID_ARG


def test_null_arguments_rejected_on_host():
    L = mjp.lib()
    assert L.mjp_plan_create_csr(None, None, None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_plan_create_stencil(None, None, None) == mjp.MJP_E_INVALID_ARG
    t = np.array([1.0])
    assert L.mjp_expv(None, None, 1, t.ctypes.data, None, None, None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_expv_batched(-1, None, None, None, None, None, None, None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_expv_batched(0, None, None, None, None, None, None, None) == mjp.MJP_OK
    assert mjp.mjp_last_error() == ""
    L.mjp_plan_destroy(None)   # accepted
    assert L.mjp_plan_n(None) == 0


def test_no_device_reports_device_error():
    """A valid operator on a machine without a GPU fails with MJP_E_DEVICE
    (the host checks all passed first)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert status_of(mjp.mjp_plan_create_csr, *GOOD) == mjp.MJP_E_DEVICE


def _ll_status(model=1, B=1, T=(1.0,), recs=((0, 1, 1, 1),), x0=(0, 0), **opts):
    obs = mjp.make_obs(np.asarray(T, float), np.asarray(recs, np.int32).reshape(-1, 4), x0)
    L = mjp.lib()
    o = mjp.mjp_opts_default(**opts)
    dummy = np.zeros(8)
    return L.mjp_loglik(model, B, dummy.ctypes.data, dummy.ctypes.data, ctypes.byref(obs), ctypes.byref(o),
                        dummy.ctypes.data, None, None)


@pytest.mark.parametrize("kw,expect", [
    (dict(model=5), mjp.MJP_E_INVALID_ARG),
    (dict(B=-1), mjp.MJP_E_INVALID_ARG),
    (dict(T=()), mjp.MJP_E_INVALID_ARG),
    (dict(T=(1.0, -2.0)), mjp.MJP_E_INVALID_ARG),
    (dict(recs=((3, 1, 1, 1),)), mjp.MJP_E_INVALID_ARG),       # time index out of range
    (dict(recs=((0, 1, 1, 0),)), mjp.MJP_E_INVALID_ARG),       # count 0
    (dict(recs=((0, -1, 1, 1),)), mjp.MJP_E_INVALID_ARG),      # negative state
    (dict(model=0, recs=((0, 1, 1, 1),)), mjp.MJP_E_INVALID_ARG),  # BD with x2 != 0
    (dict(x0=(-1, 0)), mjp.MJP_E_INVALID_ARG),
    (dict(truncation=mjp.MJP_LEAKY, renorm_every=0), mjp.MJP_E_UNSUPPORTED),
    (dict(tol=2.0), mjp.MJP_E_INVALID_ARG),
    (dict(B=0), mjp.MJP_OK),
])
def test_loglik_validation(kw, expect):
    assert _ll_status(**kw) == expect


def test_loglik_capacity():
    assert mjp.mjp_loglik_max_states() == 40000


def test_loglik_shape_table():
    """Every shape's capacity is min(T*C, 40000) in at most 160 KB of LDS
    (plus the weight/window scratch); every size class has its default
    shape (T = 1024, so every record count fits) and at least two others."""
    shapes = mjp.mjp_loglik_shapes()
    limits = mjp.mjp_loglik_class_limits()
    assert limits == sorted(limits) and limits[-1] == mjp.mjp_loglik_max_states()
    assert mjp.lib().mjp_loglik_class_limit(-1) == 0 and mjp.lib().mjp_loglik_class_limit(4) == 0
    for sh in shapes:
        assert sh["max_states"] == min(sh["threads"] * sh["cells"], 40000)
        assert sh["threads"] % 64 == 0 and sh["lds_bytes"] <= 4 * 40000 + 4096
    for lim in limits:
        fit = [i for i, sh in enumerate(shapes) if sh["max_states"] >= lim]
        assert len(fit) >= 3 and any(shapes[i]["threads"] == 1024 for i in fit)
    out = mjp.mjp_ll_shape()
    assert mjp.lib().mjp_loglik_shape(len(shapes), ctypes.byref(out)) == mjp.MJP_E_INVALID_ARG
    assert mjp.lib().mjp_loglik_shape(-1, ctypes.byref(out)) == mjp.MJP_E_INVALID_ARG


@pytest.mark.parametrize("ids", [[0, 0, 0, 99], [-2, -1, -1, -1], [0, 0, 0, 8]])  # out of range; too small for class 3
def test_loglik_set_shapes_validation(ids):
    assert status_of(mjp.mjp_loglik_set_shapes, 1, ids) == mjp.MJP_E_INVALID_ARG
    assert status_of(mjp.mjp_loglik_set_shapes, 7, [-1] * 4) == mjp.MJP_E_INVALID_ARG


def test_jump_probs_validation():
    """Host checks of mjp_jump_probs: the mjp_loglik checks, plus records of
    count 1 only."""
    L = mjp.lib()
    o = mjp.mjp_opts_default()
    d = np.zeros(8)
    def st(recs, model=0, B=1):
        obs = mjp.make_obs(np.asarray([1.0]), np.asarray(recs, np.int32).reshape(-1, 4), (0, 0))
        return L.mjp_jump_probs(model, B, d.ctypes.data, d.ctypes.data, ctypes.byref(obs), d.ctypes.data,
                                ctypes.byref(o), d.ctypes.data, None, None)
    assert st([[0, 1, 0, 2]]) == mjp.MJP_E_INVALID_ARG          # count 2
    assert st([[0, 1, 1, 1]]) == mjp.MJP_E_INVALID_ARG          # BD with x2 != 0
    assert st([[0, 1, 0, 1]], model=7) == mjp.MJP_E_INVALID_ARG
    assert st([[0, 1, 0, 1]], B=0) == mjp.MJP_OK


def test_loglik_tune_validation():
    obs = mjp.make_obs(np.asarray([1.0]), np.asarray([[0, 1, 1, 1]], np.int32), (0, 0))
    o = mjp.mjp_opts_default()
    d = np.zeros(8)
    L = mjp.lib()
    args = (ctypes.byref(obs), ctypes.byref(o), d.ctypes.data, None)
    assert L.mjp_loglik_tune(1, 1, d.ctypes.data, d.ctypes.data, *args, 0, None, None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_loglik_tune(1, 0, d.ctypes.data, d.ctypes.data, *args, 2, None, None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_loglik_tune(1, 1, None, d.ctypes.data, *args, 2, None, None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_loglik_tune(9, 1, d.ctypes.data, d.ctypes.data, *args, 2, None, None) == mjp.MJP_E_INVALID_ARG


@pytest.mark.parametrize("cfg", [(0, 256, 3), (17, 256, 3), (4, 100, 3), (4, 1024, 3), (4, 256, 0), (4, 256, 9)])
def test_surrogate_config_validation(cfg):
    c = mjp.mjp_mlp_cfg(*cfg)
    h = ctypes.c_void_p()
    assert mjp.lib().mjp_surrogate_create(ctypes.byref(c), 0, ctypes.byref(h)) == mjp.MJP_E_INVALID_ARG
    assert h.value is None


def test_surrogate_null_handles():
    L = mjp.lib()
    assert L.mjp_surrogate_num_params(None) == 0
    L.mjp_surrogate_destroy(None)
    assert L.mjp_surrogate_infer(None, None, 0, None, None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_surrogate_grad(None, None, None, 1, None, None, None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_surrogate_load(None, None) == mjp.MJP_E_INVALID_ARG


def test_surrogate_load_rejects_foreign_file(tmp_path):
    p = tmp_path / "x.bin"
    p.write_bytes(b"NOTASURROGATE" * 4)
    h = ctypes.c_void_p()
    assert mjp.lib().mjp_surrogate_load(str(p).encode(), ctypes.byref(h)) == mjp.MJP_E_INVALID_ARG


@pytest.mark.parametrize("kw,expect", [
    (dict(kappa=1), mjp.MJP_E_INVALID_ARG),
    (dict(kappa=33), mjp.MJP_E_INVALID_ARG),
    (dict(dt_factor=0.0), mjp.MJP_E_INVALID_ARG),
    (dict(dt_factor=float("nan")), mjp.MJP_E_INVALID_ARG),
    (dict(variant=3), mjp.MJP_E_INVALID_ARG),
    (dict(variant=-1), mjp.MJP_E_INVALID_ARG),
])
def test_krylov_option_validation(kw, expect):
    assert status_of(mjp.mjp_krylov_create, *GOOD, mjp.mjp_krylov_opts_default(**kw)) == expect


def test_krylov_operator_validation():
    bad = _csr([0, 2, 4], [0, 1, 0, 1], [-1.0, 1.0, -2.0, 2.0])  # negative off-diagonal rate
    assert status_of(mjp.mjp_krylov_create, *bad) == mjp.MJP_E_NOT_GENERATOR
    off = _csr([0, 2, 4], [0, 1, 0, 1], [-1.0, 1.5, 2.0, -2.0])  # row 0 sums to 0.5
    assert status_of(mjp.mjp_krylov_create, *off) == mjp.MJP_E_NOT_GENERATOR
    L = mjp.lib()
    assert L.mjp_krylov_expv(None, None, 1, None, None, None, None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_krylov_n(None) == 0
    L.mjp_krylov_destroy(None)
    o = mjp.mjp_krylov_opts_default()
    assert o.kappa == 20 and o.dt_factor == 2.0


def test_krylov_no_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert status_of(mjp.mjp_krylov_create, *GOOD) == mjp.MJP_E_DEVICE


@pytest.mark.parametrize("channels,kw,expect", [
    ([], {}, mjp.MJP_E_INVALID_ARG),                                   # no channel
    ([GOOD] * 9, {}, mjp.MJP_E_INVALID_ARG),                           # more than 8
    ([GOOD, _csr([0, 1], [0], [0.0])], {}, mjp.MJP_E_INVALID_ARG),      # sizes differ
    ([GOOD], dict(dt_factor=0.0), mjp.MJP_E_INVALID_ARG),
    ([GOOD], dict(dt_factor=float("inf")), mjp.MJP_E_INVALID_ARG),
    ([GOOD, _csr([0, 2, 4], [0, 1, 0, 1], [-1.0, 1.0, -2.0, 2.0])], {}, mjp.MJP_E_NOT_GENERATOR),
    ([_csr([0, 2, 4], [0, 1, 0, 1], [-1.0, 1.5, 2.0, -2.0])], {}, mjp.MJP_E_NOT_GENERATOR),
])
def test_rk4_create_validation(channels, kw, expect):
    assert status_of(mjp.mjp_rk4_create, channels, mjp.mjp_rk4_opts_default(**kw)) == expect


def test_rk4_null_handles_and_defaults():
    L = mjp.lib()
    assert L.mjp_rk4_expv(None, None, 1, None, None, None, None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_rk4_set_schedule(None, 0, 1, None, None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_rk4_n(None) == 0
    L.mjp_rk4_destroy(None)
    assert mjp.mjp_rk4_opts_default().dt_factor == 1.0


def test_rk4_no_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert status_of(mjp.mjp_rk4_create, [GOOD, GOOD]) == mjp.MJP_E_DEVICE
    assert status_of(mjp.mjp_rk4_create_stencil, mjp.make_model(1, [1.0, 1.0, 1.0, 1.0], [4, 3])) == \
        mjp.MJP_E_DEVICE


@pytest.mark.parametrize("model,theta,dims,kw,expect", [
    (2, [1.0] * 4, [5, 2], {}, mjp.MJP_E_INVALID_ARG),            # two-state needs dims[1] = 1
    (3, [1.0, 1.0, 1.0, 1.0, 1.0, -2.0], [5, 4], {}, mjp.MJP_E_INVALID_ARG),  # negative binding rate
    (0, [1.0, 1.0], [0, 1], {}, mjp.MJP_E_INVALID_ARG),            # empty grid
    (0, [1.0, 1.0], [5, 2], {}, mjp.MJP_E_INVALID_ARG),            # birth-death needs dims[1] = 1
    (1, [1.0, -1.0, 1.0, 1.0], [5, 4], {}, mjp.MJP_E_INVALID_ARG),  # negative rate
    (1, [1.0, float("nan"), 1.0, 1.0], [5, 4], {}, mjp.MJP_E_INVALID_ARG),
    (1, [1.0] * 4, [5, 4], dict(dt_factor=-1.0), mjp.MJP_E_INVALID_ARG),
    (7, [1.0] * 4, [5, 4], {}, mjp.MJP_E_INVALID_ARG),             # unknown model
])
def test_rk4_create_stencil_validation(model, theta, dims, kw, expect):
    assert status_of(mjp.mjp_rk4_create_stencil, mjp.make_model(model, theta, dims),
                     mjp.mjp_rk4_opts_default(**kw)) == expect


def test_rk4_create_stencil_null_arguments():
    L = mjp.lib()
    o = mjp.mjp_rk4_opts_default()
    m = mjp.make_model(1, [1.0] * 4, [3, 3])
    h = ctypes.c_void_p()
    assert L.mjp_rk4_create_stencil(None, ctypes.byref(o), ctypes.byref(h)) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_rk4_create_stencil(ctypes.byref(m), None, ctypes.byref(h)) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_rk4_create_stencil(ctypes.byref(m), ctypes.byref(o), None) == mjp.MJP_E_INVALID_ARG


@pytest.mark.parametrize("model,dims", [(2, [0, 1]), (2, [5, 2]), (3, [0, 4]), (3, [4, 0])])
def test_new_model_dims_validation(model, dims):
    m = mjp.make_model(model, [1.0] * 6, dims)
    assert status_of(mjp.mjp_model_csr, m) == mjp.MJP_E_INVALID_ARG


def test_stencil_plans_take_gene_state_models():
    """Stencil plans cover the two-state and autoregulatory models: their
    host checks pass (without a GPU the only failure left is the device
    lookup), and bad dims are rejected before that."""
    for model, dims in ((2, [10, 1]), (3, [4, 5])):
        st = status_of(mjp.mjp_plan_create_stencil, mjp.make_model(model, [1.0] * 6, dims))
        assert st in (mjp.MJP_OK, mjp.MJP_E_DEVICE), st
    for model, dims in ((2, [0, 1]), (3, [4, 0])):
        assert status_of(mjp.mjp_plan_create_stencil, mjp.make_model(model, [1.0] * 6, dims)) == mjp.MJP_E_INVALID_ARG


def test_noalloc_loglik_rejects_oversize_on_the_host():
    """mjp_loglik_noalloc sizes its tables on the host and refuses a call
    whose tables exceed the fixed array (MJP_E_WORKSPACE) before touching
    the GPU (the device pointers below are never dereferenced)."""
    cap = mjp.mjp_loglik_noalloc_capacity()
    assert cap == 6 << 20
    assert mjp.mjp_loglik_noalloc_bytes(-1, 1, 1) == -1
    a, b = mjp.mjp_loglik_noalloc_bytes(100, 20, 1000), mjp.mjp_loglik_noalloc_bytes(200, 20, 1000)
    assert b - a >= 100 * (24 * 20 + 8)
    assert mjp.mjp_loglik_noalloc_bytes(8192, 20, 1000) <= cap < mjp.mjp_loglik_noalloc_bytes(20000, 20, 1000)
    T = np.linspace(0.5, 10, 20)
    recs = np.array([[0, 1, 2, 1]], np.int32)
    obs = mjp.make_obs(T, recs, (0, 0))
    fake = ctypes.c_void_p(0x1000)
    st = mjp.lib().mjp_loglik_noalloc(1, 20000, fake, fake, ctypes.byref(obs), ctypes.byref(mjp.mjp_opts_default()),
                                      fake, None, None)
    assert st == mjp.MJP_E_WORKSPACE
    assert "scratch" in mjp.mjp_last_error()


def test_sampler_rejects_bad_configuration_on_the_host():
    L = mjp.lib()
    obs = mjp.make_obs([1.0], [[0, 3, 0, 1]])
    opts = mjp.mjp_opts_default()
    h = ctypes.c_void_p()
    cfg = mjp.mjp_sampler_cfg_default(model=mjp.MJP_MODEL_BD, dims=(50, 1), chains=8)
    assert L.mjp_sampler_create(None, ctypes.byref(obs), ctypes.byref(opts), ctypes.byref(h)) == mjp.MJP_E_INVALID_ARG
    for bad in (dict(model=7), dict(chains=0), dict(dims=(0, 1)), dict(prior_sigma=0.0),
                dict(prior_mu=float("nan"))):
        c = mjp.mjp_sampler_cfg_default(**{**dict(model=mjp.MJP_MODEL_BD, dims=(50, 1), chains=8), **bad})
        assert L.mjp_sampler_create(ctypes.byref(c), ctypes.byref(obs), ctypes.byref(opts),
                                    ctypes.byref(h)) == mjp.MJP_E_INVALID_ARG, bad
    empty = mjp.make_obs([1.0], np.zeros((0, 4), np.int32))
    assert L.mjp_sampler_create(ctypes.byref(cfg), ctypes.byref(empty), ctypes.byref(opts),
                                ctypes.byref(h)) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_sampler_set_proposal(None, None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_sampler_run(None, 1, None, 0, None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_philox_fill(1, 0, 0, 0, -1, None, None) == mjp.MJP_E_INVALID_ARG


def _cache_file(tmp_path, gpu="gfx950 256 AMD_Instinct_MI355X", table=None, models=None):
    """A shape-cache file in the library's text format (the format is stated
    in include/mjp.h beside mjp_loglik_save_shapes)."""
    if table is None:
        table = " ".join([str(len(mjp.mjp_loglik_shapes()))] + [str(c) for c in mjp.mjp_loglik_class_limits()])
    models = models or [[-1, -1, -1, -1]] * 4
    lines = ["mjp-loglik-shapes 1", f"gpu {gpu}", f"table {table}"]
    lines += [f"model {m} " + " ".join(str(v) for v in ids) for m, ids in enumerate(models)]
    p = tmp_path / "shapes.txt"
    p.write_text("\n".join(lines) + "\n")
    return str(p)


def test_shape_cache_rejects_bad_files_on_the_host(tmp_path):
    L = mjp.lib()
    assert L.mjp_loglik_save_shapes(None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_loglik_load_shapes(None) == mjp.MJP_E_INVALID_ARG
    assert L.mjp_loglik_load_shapes(str(tmp_path / "missing").encode()) == mjp.MJP_E_INVALID_ARG
    junk = tmp_path / "junk"
    junk.write_text("not a cache\n")
    assert L.mjp_loglik_load_shapes(str(junk).encode()) == mjp.MJP_E_INVALID_ARG
    # a shape that cannot hold its class, a shape id out of range, a truncated file
    assert status_of(mjp.mjp_loglik_load_shapes, _cache_file(tmp_path, models=[[0, 0, 0, 8]] * 4)) == \
        mjp.MJP_E_INVALID_ARG
    assert status_of(mjp.mjp_loglik_load_shapes, _cache_file(tmp_path, models=[[99, -1, -1, -1]] * 4)) == \
        mjp.MJP_E_INVALID_ARG
    p = _cache_file(tmp_path)
    with open(p) as f:
        head = f.readlines()[:5]
    open(p, "w").writelines(head)
    assert status_of(mjp.mjp_loglik_load_shapes, p) == mjp.MJP_E_INVALID_ARG
    # a valid cache with a long tail of extra lines (reading stops at the eighth)
    p = _cache_file(tmp_path)
    with open(p, "a") as f:
        f.write("x\n" * 100000)
    assert status_of(mjp.mjp_loglik_load_shapes, p) == mjp.MJP_E_INVALID_ARG
    # written by a build with another shape table: refused before any device query
    assert status_of(mjp.mjp_loglik_load_shapes, _cache_file(tmp_path, table="3 1 2 3 4")) == mjp.MJP_E_UNSUPPORTED


def test_shape_cache_needs_a_device_for_its_key(tmp_path):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert status_of(mjp.mjp_loglik_load_shapes, _cache_file(tmp_path)) == mjp.MJP_E_DEVICE
    assert status_of(mjp.mjp_loglik_save_shapes, str(tmp_path / "out.txt")) == mjp.MJP_E_DEVICE
