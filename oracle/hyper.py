"""Hold-out loss of the FSDA ratings and its hypergradient -- TEST INFRASTRUCTURE ONLY.

For a held-out set of rows (indices ho, targets y_ho) and every shift,

    H(beta, alpha) = 1/2 || X_ho w - y_ho ||^2 / n_ho,   w = A(beta, alpha)^{-1} b,

with the ratings X w of Alg. 7 (uncentred) and A the operator of Alg. 7, step 4
(b does not depend on beta or alpha).  A is symmetric, so one adjoint solve per
shift gives both derivatives:

    A lambda = X_ho^T (X_ho w - y_ho) / n_ho,
    dH/d log beta = -beta <lambda, w>,
    dH/d alpha    = -<lambda, (dA/dalpha) w>,  dA/dalpha = X^T [L - (P_l - 1_l 1_l^T / l)] X,

A being affine in alpha.  Built from the CG oracle (oracle.solve, oracle.apply,
oracle.project); pinned against central differences of dense solves.
"""
from __future__ import annotations

import numpy as np

import oracle


def xt(pb, v: np.ndarray) -> np.ndarray:
    """X^T v (uncentred): the centred product plus mu_l sum(v)."""
    return oracle.xct(pb, v) + oracle.mean_labeled(pb) * float(np.sum(v))


def loss(pb, W: np.ndarray, ho_idx, ho_y) -> np.ndarray:
    S = oracle.project(pb, W)[:, ho_idx]
    r = S - np.asarray(ho_y, dtype=np.float64)[None, :]
    return 0.5 * (r * r).sum(axis=1) / len(ho_idx)


def adjoint_rhs(pb, W: np.ndarray, ho_idx, ho_y) -> np.ndarray:
    S = oracle.project(pb, W)[:, ho_idx]
    G = np.zeros_like(W)
    for s in range(W.shape[0]):
        e = np.zeros(pb.n)
        e[ho_idx] = (S[s] - np.asarray(ho_y, dtype=np.float64)) / len(ho_idx)
        G[s] = xt(pb, e)
    return G


def gradients(pb, betas, ho_idx, ho_y, alpha=None, rtol: float = 1e-13, maxit: int = 100000):
    """(loss [S], dH/dlog beta [S], dH/dalpha [S], W [S, d], Lambda [S, d])."""
    a = pb.alpha if alpha is None else alpha
    betas = np.asarray(betas, dtype=np.float64)
    W, *_ = oracle.solve(pb, betas=betas, rtol=rtol, maxit=maxit, alpha=a)
    G = adjoint_rhs(pb, W, ho_idx, ho_y)
    Lam = np.zeros_like(W)
    for s, beta in enumerate(betas):
        Lam[s] = oracle.solve(pb, betas=[beta], rtol=rtol, maxit=maxit, b=G[s], alpha=a)[0][0]
    dlogb = np.array([-beta * Lam[s] @ W[s] for s, beta in enumerate(betas)])
    dalpha = np.array([-(Lam[s] @ (oracle.apply(pb, 0.0, W[s], alpha=1.0) - oracle.apply(pb, 0.0, W[s], alpha=0.0)))
                       for s in range(betas.size)])
    return loss(pb, W, ho_idx, ho_y), dlogb, dalpha, W, Lam
