"""Pins of the spectral-analysis solve (Alg. sasda) in the CPU oracle.

The oracle runs plain CG per shift on Cl^T M + beta I_N, applied as printed
(one-sided).  These tests tie it to things it does not compute itself: dense
LU of the explicitly built matrix, closed forms at alpha = 0 and for an empty
graph, the equivalence with the feature-space solve when X = I_N (the remark of
Sec. 4.2 that the SA phase is an SDA problem with the identity as data
matrix), the annihilated all-ones direction, and the printed right-hand side.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from oracle import dense


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def identity_data(pb):
    """The same problem with X = I_N (d = n)."""
    return dataclasses.replace(pb, d=pb.n, x_rowptr=np.arange(pb.n + 1, dtype=np.int32),
                               x_col=np.arange(pb.n, dtype=np.int32))


@pytest.mark.parametrize("seed", [1, 2])
@pytest.mark.parametrize("alpha", [0.3, 0.5, 1.0])
def test_sa_vs_dense_lu(seed, alpha):
    pb = synth.small_problem(n=60, d=40, mean_nnz=5, k=3, alpha=alpha, seed=seed)
    Z, it, rel, rc = oracle.sa_solve(pb, rtol=1e-13, maxit=5000)
    assert rc == oracle.OK
    for s, beta in enumerate(pb.betas):
        assert relerr(Z[s], dense.sa_solve_dense(pb, beta)) < 1e-9, (s, beta)
        assert rel[s] < 1e-12


def test_sa_apply_vs_dense():
    pb = synth.small_problem(n=45, d=30, k=4, alpha=0.6, seed=4)
    z = synth.normal(pb.n, seed=3, stream=2)
    for beta in (0.0, 0.2, 5.0):
        q = oracle.sa_apply(pb, beta, z)
        assert np.abs(q - dense.sa_operator(pb, beta) @ z).max() < 1e-12 * np.abs(q).max()


@pytest.mark.parametrize("beta", [1e-3, 0.1, 10.0])
def test_sa_alpha0_closed_form(beta):
    """alpha = 0: the operator acts on the labeled block only, as I - 1 1^T / l there; y_c is orthogonal
    to 1_l, so the labeled ratings are y_c / (1 + beta) and the unlabeled ones are exactly 0."""
    pb = synth.small_problem(n=80, d=40, k=3, n_lab=15, alpha=0.0, seed=6)
    Z, *_ = oracle.sa_solve(pb, betas=[beta], rtol=1e-14, maxit=100)
    g = oracle.sa_rhs(pb)
    unl = np.setdiff1d(np.arange(pb.n), pb.lab_idx)
    assert np.all(Z[0, unl] == 0.0)
    assert np.allclose(Z[0, pb.lab_idx], g[pb.lab_idx] / (1.0 + beta), rtol=1e-12, atol=0)


def test_sa_empty_graph_alpha1_gives_g_over_beta():
    pb = synth.small_problem(n=30, d=25, alpha=1.0, seed=3)
    pb.s_rowptr = np.zeros(pb.n + 1, dtype=np.int32)
    pb.s_col = np.zeros(0, dtype=np.int32)
    Z, it, rel, rc = oracle.sa_solve(pb, rtol=1e-14, maxit=10)
    g = oracle.sa_rhs(pb)
    for s, beta in enumerate(pb.betas):
        assert np.allclose(Z[s], g / beta, rtol=1e-15, atol=0)


@pytest.mark.parametrize("alpha", [0.0, 0.4, 1.0])
def test_sa_equals_feature_space_solve_with_identity_data(alpha):
    pb = synth.small_problem(n=70, d=50, mean_nnz=6, k=3, alpha=alpha, seed=11)
    Z, *_ = oracle.sa_solve(pb, rtol=1e-13, maxit=5000)
    W, *_ = oracle.solve(identity_data(pb), rtol=1e-13, maxit=5000)
    for s in range(pb.betas.size):
        assert relerr(Z[s], W[s]) < 1e-9
    assert np.allclose(oracle.rhs(identity_data(pb)), oracle.sa_rhs(pb), rtol=0, atol=1e-15)


@pytest.mark.parametrize("alpha", [0.0, 0.5, 1.0])
def test_sa_ones_direction_annihilated_and_ratings_sum_to_zero(alpha):
    pb = synth.small_problem(n=50, d=40, k=3, alpha=alpha, seed=9)
    ones = np.ones(pb.n)
    assert np.abs(oracle.sa_apply(pb, 0.7, ones) - 0.7 * ones).max() < 1e-13
    Z, *_ = oracle.sa_solve(pb, rtol=1e-13, maxit=5000)
    for s in range(pb.betas.size):
        assert abs(Z[s].sum()) < 1e-10 * np.abs(Z[s]).sum()


def test_sa_printed_rhs_is_multiple_of_centred_labels():
    pb = synth.small_problem(n=60, d=30, k=3, n_lab=20, alpha=0.5, seed=12)
    r = synth.uniform(pb.n, -1.0, 1.0, seed=2, stream=5)
    g = oracle.sa_rhs(pb, r)
    assert np.allclose(g, dense.sa_rhs(pb, r), rtol=0, atol=1e-14)
    yc = oracle.sa_rhs(pb)
    lab = pb.lab_idx
    ratio = g[lab] / yc[lab]
    assert np.allclose(ratio, ratio[0], rtol=1e-12)
    # the multiple is half the difference of the class means of r over the labeled rows
    y = np.asarray(pb.lab_y)
    half = 0.5 * (r[lab][y > 0].mean() - r[lab][y < 0].mean())
    assert abs(ratio[0] - half) < 1e-12 * abs(half)
    assert np.all(g[np.setdiff1d(np.arange(pb.n), lab)] == 0.0)
