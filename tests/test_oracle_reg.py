"""Pins of the regression-phase solve (X^T X + beta I) w = X^T z in the CPU oracle."""
import numpy as np
import pytest

import oracle
import synth
from oracle import dense


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("seed", [1, 2])
def test_reg_vs_dense_lu_and_svd(seed):
    pb = synth.small_problem(n=50, d=40, mean_nnz=6, k=2, seed=seed)
    z = synth.normal(pb.n, seed=seed, stream=7)
    betas = np.array([1e-3, 0.1, 1.0, 30.0])
    W, it, rel, rc = oracle.reg_solve(pb, z, betas, rtol=1e-13, maxit=5000)
    assert rc == oracle.OK
    for s, beta in enumerate(betas):
        assert relerr(W[s], dense.reg_solve_dense(pb, beta, z)) < 1e-9
        assert relerr(W[s], dense.reg_solve_svd(pb, beta, z)) < 1e-9
        assert rel[s] < 1e-12


def test_reg_large_shift_asymptote():
    """w = X^T z / beta - X^T X X^T z / beta^2 + O(beta^-3)."""
    pb = synth.small_problem(n=40, d=30, mean_nnz=5, seed=4)
    z = synth.normal(pb.n, seed=1, stream=1)
    X = dense.dense_x(pb)
    b = X.T @ z
    beta = 1e6
    W, *_ = oracle.reg_solve(pb, z, [beta], rtol=1e-15, maxit=100)
    approx = b / beta - X.T @ (X @ b) / beta ** 2
    assert np.abs(W[0] - approx).max() < 1e-3 * np.abs(b / beta ** 2).max() * np.abs(X.T @ X).max() + 1e-300


def test_reg_normal_equations_residual():
    pb = synth.small_problem(n=70, d=90, mean_nnz=7, seed=6)
    z = synth.normal(pb.n, seed=2, stream=4)
    W, *_ = oracle.reg_solve(pb, z, [0.05], rtol=1e-13, maxit=5000)
    X = dense.dense_x(pb)
    r = X.T @ z - (X.T @ (X @ W[0]) + 0.05 * W[0])
    assert np.linalg.norm(r) < 1e-12 * np.linalg.norm(X.T @ z)
