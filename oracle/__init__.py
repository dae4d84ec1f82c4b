"""CPU oracle for the FSDA multi-shift solve -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never links, imports or
calls anything here, and nothing here uses the GPU library.

Contents
  * ``fsda_oracle.c`` (via :func:`solve`, :func:`apply`, :func:`rhs`, ...):
    plain FP64 per-shift conjugate gradient (Alg. 2) on the centred,
    regularised SDA system of Alg. 7, with both centred products of Sec. 3.2.3
    written out.  OpenMP, fixed-order reductions.
  * the same file's spectral-analysis variant (Alg. sasda; :func:`sa_solve`,
    :func:`sa_apply`, :func:`sa_rhs`): per-shift CG in sample space on
    Cl^T M + beta I_N, the ratings being the solution itself.
  * the regression phase of the spectral-regression variants (:func:`reg_solve`):
    per-shift CG on (X^T X + beta I) w = X^T z.
  * :mod:`oracle.hyper`: the hold-out loss of the ratings and its gradient in
    log beta and alpha by one adjoint solve per shift.
  * :mod:`oracle.dense`: dense NumPy/SciPy forms (Cholesky of the operator,
    sample-space push-through, labeled-only dual ridge) used to pin the above.
  * :mod:`oracle.shifted`: the paper's shifted CG (Alg. 3) in NumPy, for the
    reading of its shift recurrences.
  * :mod:`oracle.exact`: exact rational arithmetic on micro problems.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
from scipy import linalg as scipy_linalg

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, NOT_CONVERGED, E_ARG, E_LABELS, E_BREAKDOWN = 0, 1, -1, -3, -5


def build(force: bool = True) -> str:
    """Compile ``fsda_oracle.c`` into ``liboracle.so``."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               os.path.join(_HERE, "fsda_oracle.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int64),
                ("x_rowptr", ctypes.c_void_p), ("x_col", ctypes.c_void_p),
                ("s_rowptr", ctypes.c_void_p), ("s_col", ctypes.c_void_p),
                ("n_lab", ctypes.c_int64), ("lab_idx", ctypes.c_void_p), ("lab_y", ctypes.c_void_p),
                ("alpha", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        pp = ctypes.POINTER(_Problem)
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = None
        lib.orc_max_threads.restype = ctypes.c_int
        lib.orc_mean_labeled.argtypes = [pp, P]
        lib.orc_apply.argtypes = [pp, ctypes.c_double, P, P]
        lib.orc_m_apply.argtypes = [pp, P, P]
        lib.orc_xct.argtypes = [pp, P, P]
        lib.orc_rhs.argtypes = [pp, P, P]
        lib.orc_solve.argtypes = [pp, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int, P, P, P, P]
        lib.orc_project.argtypes = [pp, P, ctypes.c_int, P]
        lib.orc_sa_rhs.argtypes = [pp, P, P]
        lib.orc_sa_apply.argtypes = [pp, ctypes.c_double, P, P]
        lib.orc_sa_solve.argtypes = [pp, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int, P, P, P]
        lib.orc_reg_solve.argtypes = [pp, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int, P, P, P]
        for f in (lib.orc_mean_labeled, lib.orc_apply, lib.orc_m_apply, lib.orc_xct, lib.orc_rhs,
                  lib.orc_solve, lib.orc_project, lib.orc_sa_rhs, lib.orc_sa_apply, lib.orc_sa_solve, lib.orc_reg_solve):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


class _Bound:
    """Keeps the contiguous arrays alive while the C struct points at them."""

    def __init__(self, pb, alpha=None):
        self.x_rowptr = np.ascontiguousarray(pb.x_rowptr, dtype=np.int32)
        self.x_col = np.ascontiguousarray(pb.x_col, dtype=np.int32)
        self.s_rowptr = np.ascontiguousarray(pb.s_rowptr, dtype=np.int32)
        self.s_col = np.ascontiguousarray(pb.s_col, dtype=np.int32)
        if self.s_col.size == 0:
            self.s_col = np.zeros(1, dtype=np.int32)
        if self.x_col.size == 0:
            self.x_col = np.zeros(1, dtype=np.int32)
        self.lab_idx = np.ascontiguousarray(pb.lab_idx, dtype=np.int32)
        self.lab_y = np.ascontiguousarray(pb.lab_y, dtype=np.int8)
        a = pb.alpha if alpha is None else alpha
        self.c = _Problem(pb.n, pb.d, self.x_rowptr.ctypes.data, self.x_col.ctypes.data,
                          self.s_rowptr.ctypes.data, self.s_col.ctypes.data, self.lab_idx.size,
                          self.lab_idx.ctypes.data, self.lab_y.ctypes.data, float(a))

    @property
    def ref(self):
        return ctypes.byref(self.c)


def _check(rc, what):
    if rc < 0:
        raise RuntimeError("oracle %s failed with status %d" % (what, rc))
    return rc


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def mean_labeled(pb) -> np.ndarray:
    """mu_l = X^T 1_l / l (Alg. 7, step 3)."""
    b = _Bound(pb)
    mu = np.empty(pb.d)
    _check(_load().orc_mean_labeled(b.ref, _p(mu)), "mean_labeled")
    return mu


def apply(pb, beta: float, p: np.ndarray, alpha=None) -> np.ndarray:
    """q = (Xc^T M Xc + beta I) p."""
    b = _Bound(pb, alpha)
    p = np.ascontiguousarray(p, dtype=np.float64)
    q = np.empty(pb.d)
    _check(_load().orc_apply(b.ref, float(beta), _p(p), _p(q)), "apply")
    return q


def m_apply(pb, t: np.ndarray, alpha=None) -> np.ndarray:
    """u = ((1-alpha) P_l + alpha L) t in sample space."""
    b = _Bound(pb, alpha)
    t = np.ascontiguousarray(t, dtype=np.float64)
    u = np.empty(pb.n)
    _check(_load().orc_m_apply(b.ref, _p(t), _p(u)), "m_apply")
    return u


def xct(pb, v: np.ndarray) -> np.ndarray:
    """Xc^T v = X^T v - mu_l sum(v)."""
    b = _Bound(pb)
    v = np.ascontiguousarray(v, dtype=np.float64)
    u = np.empty(pb.d)
    _check(_load().orc_xct(b.ref, _p(v), _p(u)), "xct")
    return u


def rhs(pb, r: np.ndarray = None) -> np.ndarray:
    """Canonical b = Xc^T y_c (r is None) or the Alg. 7 right-hand side for start vector r."""
    bnd = _Bound(pb)
    out = np.empty(pb.d)
    rr = None if r is None else np.ascontiguousarray(r, dtype=np.float64)
    _check(_load().orc_rhs(bnd.ref, _p(rr), _p(out)), "rhs")
    return out


def solve(pb, betas=None, rtol: float = 1e-12, maxit: int = 100000, b: np.ndarray = None, alpha=None):
    """Per-shift CG.  Returns (W [S, d], iters [S], relres [S] (true), status)."""
    bnd = _Bound(pb, alpha)
    betas = np.ascontiguousarray(pb.betas if betas is None else betas, dtype=np.float64)
    S = betas.size
    W = np.zeros((S, pb.d))
    iters = np.zeros(S, dtype=np.int32)
    relres = np.zeros(S)
    bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
    rc = _load().orc_solve(bnd.ref, _p(bb), S, _p(betas), float(rtol), int(maxit), _p(W), _p(iters), _p(relres),
                           None)
    _check(rc, "solve")
    return W, iters, relres, rc


def solve_with_kappa(pb, betas=None, rtol: float = 1e-12, maxit: int = 100000, b: np.ndarray = None, alpha=None):
    """Per-shift CG as :func:`solve`, and kappa-hat per shift: the condition estimate of
    A(beta_s) from that shift's CG run (Sec. 3.2.1).  CG's coefficients a_i, b_i define
    the Lanczos tridiagonal T (diagonal 1/a_i + b_{i-1}/a_{i-1}, off-diagonal
    sqrt(b_i)/a_i), whose extreme eigenvalues (Ritz values) approach those of A on the
    Krylov space of b.  Returns (W [S, d], iters [S], relres [S], status, kappa [S],
    ritz_min [S], ritz_max [S])."""
    bnd = _Bound(pb, alpha)
    betas = np.ascontiguousarray(pb.betas if betas is None else betas, dtype=np.float64)
    S = betas.size
    W = np.zeros((S, pb.d))
    iters = np.zeros(S, dtype=np.int32)
    relres = np.zeros(S)
    rec = np.zeros((S, 2 * int(maxit)))
    bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
    rc = _load().orc_solve(bnd.ref, _p(bb), S, _p(betas), float(rtol), int(maxit), _p(W), _p(iters), _p(relres),
                           _p(rec))
    _check(rc, "solve")
    kap, lo, hi = np.full(S, np.nan), np.full(S, np.nan), np.full(S, np.nan)
    for s in range(S):
        k = int(iters[s])
        if k == 0:
            continue
        a, bcoef = rec[s, 0:2 * k:2], rec[s, 1:2 * k:2]
        diag = 1.0 / a
        diag[1:] += bcoef[:-1] / a[:-1]
        off = np.sqrt(bcoef[:-1]) / a[:-1]
        ev = scipy_linalg.eigvalsh_tridiagonal(diag, off) if k > 1 else diag
        lo[s], hi[s] = ev[0], ev[-1]
        kap[s] = ev[-1] / ev[0]
    return W, iters, relres, rc, kap, lo, hi


def lanczos_condition(pb, betas=None, rtol: float = 1e-10, maxit: int = 20000, b: np.ndarray = None, alpha=None):
    """kappa-hat per shift from the CG run of that shift (see :func:`solve_with_kappa`).
    Returns (kappa [S], ritz_min [S], ritz_max [S], iters [S])."""
    W, iters, relres, rc, kap, lo, hi = solve_with_kappa(pb, betas, rtol, maxit, b, alpha)
    return kap, lo, hi, iters


def project(pb, W: np.ndarray) -> np.ndarray:
    """Ratings s = X w per shift (Alg. 7 return value)."""
    bnd = _Bound(pb)
    W = np.ascontiguousarray(np.atleast_2d(W), dtype=np.float64)
    out = np.empty((W.shape[0], pb.n))
    _check(_load().orc_project(bnd.ref, _p(W), W.shape[0], _p(out)), "project")
    return out


def sa_rhs(pb, r: np.ndarray = None, alpha=None) -> np.ndarray:
    """Alg. sasda right-hand side: y_c (r is None) or [W 0; 0 0](r - 1 <1_l, r>/l)."""
    bnd = _Bound(pb, alpha)
    out = np.empty(pb.n)
    rr = None if r is None else np.ascontiguousarray(r, dtype=np.float64)
    _check(_load().orc_sa_rhs(bnd.ref, _p(rr), _p(out)), "sa_rhs")
    return out


def sa_apply(pb, beta: float, z: np.ndarray, alpha=None) -> np.ndarray:
    """q = (Cl^T M + beta I_N) z (Alg. sasda, step 4)."""
    bnd = _Bound(pb, alpha)
    z = np.ascontiguousarray(z, dtype=np.float64)
    q = np.empty(pb.n)
    _check(_load().orc_sa_apply(bnd.ref, float(beta), _p(z), _p(q)), "sa_apply")
    return q


def sa_solve(pb, betas=None, rtol: float = 1e-12, maxit: int = 100000, g: np.ndarray = None, alpha=None):
    """Alg. sasda per shift.  Returns (Z [S, n] = ratings, iters [S], relres [S] (true), status)."""
    bnd = _Bound(pb, alpha)
    betas = np.ascontiguousarray(pb.betas if betas is None else betas, dtype=np.float64)
    S = betas.size
    Z = np.zeros((S, pb.n))
    iters = np.zeros(S, dtype=np.int32)
    relres = np.zeros(S)
    gg = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
    rc = _load().orc_sa_solve(bnd.ref, _p(gg), S, _p(betas), float(rtol), int(maxit), _p(Z), _p(iters), _p(relres))
    _check(rc, "sa_solve")
    return Z, iters, relres, rc


def reg_solve(pb, z: np.ndarray, betas, rtol: float = 1e-12, maxit: int = 100000):
    """Regression phase: (X^T X + beta I) w = X^T z per shift.  Returns (W [S, d], iters, relres, status)."""
    bnd = _Bound(pb)
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    S = betas.size
    W = np.zeros((S, pb.d))
    iters = np.zeros(S, dtype=np.int32)
    relres = np.zeros(S)
    rc = _load().orc_reg_solve(bnd.ref, _p(z), S, _p(betas), float(rtol), int(maxit), _p(W), _p(iters), _p(relres))
    _check(rc, "reg_solve")
    return W, iters, relres, rc
