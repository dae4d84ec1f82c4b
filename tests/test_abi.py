"""The C ABI library on the host: it loads, exports every declared symbol, and
rejects bad arguments before any HIP call.  No GPU needed."""
import ctypes

import numpy as np
import pytest

fsda = pytest.importorskip("paper_1709_04794_amd")


def test_every_declared_symbol_is_exported():
    names = fsda.declared_functions()
    assert {"fsda_workspace_size", "fsda_build_operator", "fsda_multishift_solve", "fsda_project", "fsda_rhs",
            "fsda_apply", "fsda_destroy_operator", "fsda_last_error"} <= set(names)
    L = fsda.lib()
    for nm in names:
        assert hasattr(L, nm), nm


def _pb(**kw):
    base = dict(n=100, d=200, x_rowptr=1, x_col=1, x_nnz=1000, s_rowptr=1, s_col=1,
                s_nnz=500, lab_idx=1, lab_y=1, n_lab=10, alpha=0.5, precision=0)
    base.update(kw)
    return fsda.Problem(**base)


def _ws(pb, ms=16, mc=32):
    size = ctypes.c_size_t(0)
    rc = fsda.lib().fsda_workspace_size(ctypes.byref(pb), ms, mc, ctypes.byref(size))
    return rc, size.value


def test_workspace_size_valid_and_monotone():
    rc, a = _ws(_pb())
    assert rc == fsda.OK and a > 0
    # large enough that the solve state, not the build scratch, sets the size
    kw = dict(n=10000, d=2000000, x_nnz=100000)
    rc, a = _ws(_pb(**kw))
    assert rc == fsda.OK
    rc, b = _ws(_pb(**kw), ms=32)
    assert rc == fsda.OK and b > a
    rc, c = _ws(_pb(**dict(kw, d=4000000)))
    assert c > a
    rc, e = _ws(_pb(**kw), mc=64)
    assert e > a


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), fsda.E_ARG),
    (dict(d=-3), fsda.E_ARG),
    (dict(alpha=1.5), fsda.E_RANGE),
    (dict(alpha=-0.1), fsda.E_RANGE),
    (dict(alpha=float("nan")), fsda.E_RANGE),
    (dict(n_lab=1), fsda.E_LABELS),
    (dict(n_lab=101), fsda.E_LABELS),
    (dict(x_nnz=2 ** 31), fsda.E_OVERFLOW),
    (dict(n=2 ** 31), fsda.E_OVERFLOW),
    (dict(x_rowptr=None), fsda.E_ARG),
    (dict(lab_y=None), fsda.E_ARG),
    (dict(precision=7), fsda.E_ARG),
])
def test_workspace_size_rejects(kw, code):
    rc, _ = _ws(_pb(**kw))
    assert rc == code
    assert len(fsda.lib().fsda_last_error()) > 0


@pytest.mark.parametrize("ms,mc", [(0, 32), (65, 32), (8, 0), (8, fsda.MAX_CHUNK + 1)])
def test_workspace_size_rejects_limits(ms, mc):
    rc, _ = _ws(_pb(), ms, mc)
    assert rc == fsda.E_RANGE


def test_build_rejects_bad_workspace_before_hip():
    pb = _pb()
    rc, need = _ws(pb)
    h = ctypes.c_void_p()
    L = fsda.lib()
    assert L.fsda_build_operator(ctypes.byref(pb), 16, 32, None, need, None, ctypes.byref(h)) == fsda.E_WORKSPACE
    assert L.fsda_build_operator(ctypes.byref(pb), 16, 32, ctypes.c_void_p(4096), need - 1, None,
                                 ctypes.byref(h)) == fsda.E_WORKSPACE
    assert L.fsda_build_operator(ctypes.byref(pb), 16, 32, ctypes.c_void_p(4096 + 8), need, None,
                                 ctypes.byref(h)) == fsda.E_WORKSPACE
    assert L.fsda_build_operator(ctypes.byref(_pb(alpha=2.0)), 16, 32, ctypes.c_void_p(4096), need, None,
                                 ctypes.byref(h)) == fsda.E_RANGE
    assert h.value is None


def test_null_handle_calls_fail_cleanly():
    L = fsda.lib()
    betas = np.array([1.0])
    it = np.zeros(1, dtype=np.int32)
    rr = np.zeros(1)
    assert L.fsda_multishift_solve(None, None, betas.ctypes.data, 1, 1e-8, 10, 0, ctypes.c_void_p(8),
                                   it.ctypes.data, rr.ctypes.data, None) == fsda.E_ARG
    assert L.fsda_project(None, ctypes.c_void_p(8), 1, ctypes.c_void_p(8), None) == fsda.E_ARG
    assert L.fsda_apply(None, 0.0, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == fsda.E_ARG
    assert L.fsda_rhs(None, None, ctypes.c_void_p(8), None) == fsda.E_ARG
    assert L.fsda_sa_rhs(None, None, ctypes.c_void_p(8), None) == fsda.E_ARG
    assert L.fsda_sa_solve(None, None, betas.ctypes.data, 1, 1e-8, 10, 0, ctypes.c_void_p(8), it.ctypes.data,
                           rr.ctypes.data, None) == fsda.E_ARG
    assert L.fsda_regression_solve(None, ctypes.c_void_p(8), betas.ctypes.data, 1, 1e-3, 10, 0, 1,
                                   ctypes.c_void_p(8), it.ctypes.data, rr.ctypes.data, None) == fsda.E_ARG
    size = ctypes.c_size_t(0)
    assert L.fsda_batch_workspace_size(None, 4, 4, 0, ctypes.byref(size)) == fsda.E_ARG
    off = np.array([0, 5], dtype=np.int64)
    assert L.fsda_multishift_solve_batch(None, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), off.ctypes.data,
                                         betas.ctypes.data, 1, 1e-8, 10, 0, ctypes.c_void_p(256), 1 << 20,
                                         ctypes.c_void_p(8), it.ctypes.data, rr.ctypes.data, None) == fsda.E_ARG
    assert b"NULL" in L.fsda_last_error()
    assert L.fsda_columns_batch_workspace_size(None, 2, 2, ctypes.byref(size)) == fsda.E_ARG
    assert L.fsda_solve_columns_batch(None, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), off.ctypes.data,
                                      betas.ctypes.data, 1, ctypes.c_void_p(8), 1e-8, 10, ctypes.c_void_p(256),
                                      1 << 20, ctypes.c_void_p(8), it.ctypes.data, rr.ctypes.data, None) == fsda.E_ARG
    loss = np.zeros(1)
    assert L.fsda_holdout_batch(None, 1, ctypes.c_void_p(8), 1, ctypes.c_void_p(8), ctypes.c_void_p(8),
                                off.ctypes.data, loss.ctypes.data, None, None) == fsda.E_ARG
    g = np.zeros(1)
    assert L.fsda_hypergradient_batch(None, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), off.ctypes.data,
                                      ctypes.c_void_p(8), ctypes.c_void_p(8), betas.ctypes.data, 1, g.ctypes.data,
                                      g.ctypes.data, None) == fsda.E_ARG
    L.fsda_destroy_operator(None)
