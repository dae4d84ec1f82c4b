"""Pins of the adjoint hypergradient (oracle.hyper) against central differences of dense solves."""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import dense, hyper


def dense_loss(pb, beta, alpha, ho, yho):
    w = dense.solve_dense(dataclasses.replace(pb, alpha=alpha), beta)
    r = dense.dense_x(pb)[ho] @ w - yho
    return 0.5 * r @ r / len(ho)


def split(pb, seed):
    rng = np.random.default_rng(seed)
    unl = np.setdiff1d(np.arange(pb.n), pb.lab_idx)
    ho = np.sort(rng.choice(unl, size=max(4, unl.size // 4), replace=False))
    yho = np.where(rng.random(ho.size) < 0.3, 1.0, -1.0)
    return ho, yho


@pytest.mark.parametrize("alpha", [0.2, 0.5, 0.9])
def test_adjoint_gradient_matches_central_differences(alpha):
    pb = synth.small_problem(n=60, d=40, mean_nnz=5, k=3, n_lab=15, alpha=alpha, seed=3)
    ho, yho = split(pb, 1)
    betas = np.array([0.03, 0.5, 4.0])
    H, dlogb, dalpha, W, Lam = hyper.gradients(pb, betas, ho, yho)
    h = 1e-4
    for s, beta in enumerate(betas):
        assert abs(H[s] - dense_loss(pb, beta, alpha, ho, yho)) < 1e-10 * max(H[s], 1e-300)
        fd_b = (dense_loss(pb, beta * np.exp(h), alpha, ho, yho) - dense_loss(pb, beta * np.exp(-h), alpha, ho, yho)) / (2 * h)
        fd_a = (dense_loss(pb, beta, alpha + h, ho, yho) - dense_loss(pb, beta, alpha - h, ho, yho)) / (2 * h)
        assert abs(dlogb[s] - fd_b) < 1e-6 * max(abs(fd_b), 1e-12), (s, dlogb[s], fd_b)
        assert abs(dalpha[s] - fd_a) < 1e-6 * max(abs(fd_a), 1e-12), (s, dalpha[s], fd_a)


def test_adjoint_rhs_is_loss_gradient_in_w():
    pb = synth.small_problem(n=50, d=30, mean_nnz=5, k=3, alpha=0.5, seed=5)
    ho, yho = split(pb, 2)
    w = synth.normal(pb.d, seed=1, stream=1)[None, :]
    G = hyper.adjoint_rhs(pb, w, ho, yho)
    h = 1e-6
    for j in (0, 7, 19):
        e = np.zeros(pb.d)
        e[j] = h
        fd = (hyper.loss(pb, w + e, ho, yho)[0] - hyper.loss(pb, w - e, ho, yho)[0]) / (2 * h)
        assert abs(G[0, j] - fd) < 1e-7 * max(1.0, abs(fd))
