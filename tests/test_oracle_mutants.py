"""Plants plausible mistakes in copies of the CPU oracle and checks the pins catch each one.

Each mutant is ``oracle/fsda_oracle.c`` with one textual change (a dropped
term, a flipped sign, a missing factor), compiled into a temporary directory
and swapped in for the real library; at least one pin must fail for it.
CPU only.
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import synth
from oracle import dense

SRC = os.path.join(os.path.dirname(oracle.__file__), "fsda_oracle.c")

FSDA_PINS = ["dense", "rhs", "annihilation"]

# Changes that must NOT matter for the pins listed with them: Sec. 3.2.3 shows
# one centred product suffices, so dropping the centring of X v leaves the
# operator unchanged; and Xc^T 1_l = 0, so the feature-space right-hand side
# Xc^T y does not need centred labels (the sample-space one, y_c itself, does:
# that change must fail the sample-space pin).
EQUIVALENT = {
    "drop_centring_in_xc": ("out[i] -= m;", "(void)m;", None),
    "labels_not_centred": ("- ybar;", "- 0.0;", FSDA_PINS),
}

MUTANTS = {
    "drop_centring_in_xct": ("out[j] -= c->mu[j] * s;", "(void)s;"),
    "laplacian_sign": ("double lt = c->deg[i] * t[i] - st;", "double lt = c->deg[i] * t[i] + st;"),
    "drop_one_minus_alpha": ("out[i] = (1.0 - a) * (c->lab[i] ? t[i] : 0.0) + a * lt;",
                             "out[i] = (c->lab[i] ? t[i] : 0.0) + a * lt;"),
    "cg_update_sign": ("w[j] -= gamma * p[j];", "w[j] += gamma * p[j];"),
    "shift_not_added": ("  xct_mul(c, c->t, q);\n  for (int64_t j = 0; j < c->pb->d; j++) q[j] += beta * p[j];",
                        "  xct_mul(c, c->t, q);\n  for (int64_t j = 0; j < c->pb->d; j++) q[j] += 0.5 * beta * p[j];"),
    "direction_uses_old_residual": ("double a = rr_new / rr;", "double a = rr / rr_new;"),
    "mu_not_divided": ("c->mu[j] /= (double)pb->n_lab;", "c->mu[j] /= 1.0;"),
    # sample-space solve (Alg. sasda) and regression phase
    "sa_drop_centring": ("q[i] = c->t[i] - (c->lab[i] ? s : 0.0) + beta * z[i];", "q[i] = c->t[i] + beta * z[i];"),
    "sa_rhs_not_orthogonalised": ("c.v[i] = r[i] - sl / (double)pb->n_lab;", "c.v[i] = r[i];"),
    "reg_shift_doubled": ("  xt_mul(c, c->v, q);\n  for (int64_t j = 0; j < c->pb->d; j++) q[j] += beta * p[j];",
                          "  xt_mul(c, c->v, q);\n  for (int64_t j = 0; j < c->pb->d; j++) q[j] += 2.0 * beta * p[j];"),
}

ALL = ["dense", "rhs", "annihilation", "sa_dense", "sa_rhs", "reg_svd"]


def _checks():
    """Quick pins; returns the list of those that hold."""
    ok = []
    pb = synth.small_problem(n=40, d=32, mean_nnz=5, k=3, alpha=0.5, seed=21, pos_frac=0.4)
    try:
        W, *_ = oracle.solve(pb, rtol=1e-13, maxit=3000)
        good = all(np.linalg.norm(W[s] - dense.solve_dense(pb, bt)) < 1e-8 * np.linalg.norm(W[s])
                   for s, bt in enumerate(pb.betas))
        if good:
            ok.append("dense")
    except RuntimeError:
        pass
    try:
        X = dense.dense_x(pb)
        y = np.asarray(pb.lab_y)
        pos, neg = pb.lab_idx[y > 0], pb.lab_idx[y < 0]
        closed = 2.0 * pos.size * neg.size / pb.lab_idx.size * (X[pos].mean(0) - X[neg].mean(0))
        if np.allclose(oracle.rhs(pb), closed, rtol=1e-12, atol=1e-12):
            ok.append("rhs")
    except RuntimeError:
        pass
    try:
        v = oracle.xct(pb, oracle.m_apply(pb, np.ones(pb.n)))
        if np.abs(v).max() < 1e-12:
            ok.append("annihilation")
    except RuntimeError:
        pass
    try:
        Z, *_ = oracle.sa_solve(pb, rtol=1e-13, maxit=3000)
        if all(np.linalg.norm(Z[s] - dense.sa_solve_dense(pb, bt)) < 1e-8 * np.linalg.norm(Z[s])
               for s, bt in enumerate(pb.betas)):
            ok.append("sa_dense")
    except RuntimeError:
        pass
    try:
        r = synth.uniform(pb.n, -1.0, 1.0, seed=3, stream=1)
        if np.allclose(oracle.sa_rhs(pb, r), dense.sa_rhs(pb, r), rtol=0, atol=1e-13):
            ok.append("sa_rhs")
    except RuntimeError:
        pass
    try:
        z = synth.normal(pb.n, seed=5, stream=2)
        Wr, *_ = oracle.reg_solve(pb, z, [0.01, 1.0], rtol=1e-13, maxit=3000)
        if all(np.linalg.norm(Wr[s] - dense.reg_solve_svd(pb, bt, z)) < 1e-8 * np.linalg.norm(Wr[s])
               for s, bt in enumerate([0.01, 1.0])):
            ok.append("reg_svd")
    except RuntimeError:
        pass
    return ok


def test_unmutated_oracle_passes_quick_pins():
    assert _checks() == ALL


def _held_with(old, new, monkeypatch):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "mut.c")
        open(path, "w").write(src.replace(old, new))
        so = os.path.join(td, "libmut.so")
        subprocess.check_call(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c99", path, "-o", so, "-lm"])
        monkeypatch.setattr(oracle, "_lib", None)
        monkeypatch.setattr(oracle, "_SO", so)
        held = _checks()
        monkeypatch.setattr(oracle, "_lib", None)
    return held


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    held = _held_with(*MUTANTS[name], monkeypatch)
    assert held != ALL, "mutant %s passed every pin" % name


@pytest.mark.parametrize("name", sorted(EQUIVALENT))
def test_equivalent_change_passes(name, monkeypatch):
    old, new, pins = EQUIVALENT[name]
    held = _held_with(old, new, monkeypatch)
    if pins is None:
        assert held == ALL
    else:
        assert [p for p in held if p in pins] == pins and held != ALL
