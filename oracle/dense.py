"""Dense forms of the SDA system for small problems -- TEST INFRASTRUCTURE ONLY.

Everything is built as explicit dense matrices straight from the paper's
definitions, so it shares no code path with the matrix-free CG in
``fsda_oracle.c``:

  X          n x d binary data matrix (Sec. 2.1)
  S, L       binary similarity matrix and Laplacian L = D - S (Sec. 2.3)
  P_l        labeled-row selector diag(1_l) (Eq. SDAeig)
  W_full     [W 0; 0 0] with W_ij = 1/N_c on the labeled class blocks (Sec. 2.1)
  C          centring matrix I_N - 1 1_l^T / l, so C X = X - 1 mu_l^T (Sec. 3.2.3)
  A(beta)    (C X)^T [(1-alpha) P_l + alpha L] X + beta I_D   (Alg. 7, step 4)
  b(r)       (C X)^T W_full X r                                (Alg. 7, step 4)

Three independent routes to the solution w = A(beta)^{-1} b:
  * dense LU of A(beta) (``solve_dense``);
  * the push-through identity (B^T M X + beta I)^{-1} B^T = B^T (M X B^T + beta I)^{-1}
    with B = C X, an n x n solve in sample space (``solve_pushthrough``);
  * for alpha = 0, the textbook ridge dual on the centred labeled rows
    w = Xlc^T (Xlc Xlc^T + beta I_l)^{-1} y_c (``solve_dual_ridge_alpha0``).
"""
from __future__ import annotations

import numpy as np


def dense_x(pb) -> np.ndarray:
    X = np.zeros((pb.n, pb.d))
    rp = np.asarray(pb.x_rowptr, dtype=np.int64)
    for i in range(pb.n):
        X[i, pb.x_col[rp[i]:rp[i + 1]]] = 1.0
    return X


def dense_s(pb) -> np.ndarray:
    S = np.zeros((pb.n, pb.n))
    rp = np.asarray(pb.s_rowptr, dtype=np.int64)
    for i in range(pb.n):
        S[i, pb.s_col[rp[i]:rp[i + 1]]] = 1.0
    return S


def laplacian(pb) -> np.ndarray:
    S = dense_s(pb)
    return np.diag(S.sum(axis=1)) - S


def labeled_selector(pb) -> np.ndarray:
    m = np.zeros(pb.n)
    m[pb.lab_idx] = 1.0
    return np.diag(m)


def between_class_weight(pb) -> np.ndarray:
    """[W 0; 0 0]: 1/N_c between two labeled rows of the same class c."""
    Wf = np.zeros((pb.n, pb.n))
    y = np.asarray(pb.lab_y)
    for cls in (1, -1):
        rows = np.asarray(pb.lab_idx)[y == cls]
        if rows.size:
            Wf[np.ix_(rows, rows)] = 1.0 / rows.size
    return Wf


def centring(pb) -> np.ndarray:
    """I_N - 1 1_l^T / l."""
    ones_l = np.zeros(pb.n)
    ones_l[pb.lab_idx] = 1.0
    return np.eye(pb.n) - np.outer(np.ones(pb.n), ones_l) / len(pb.lab_idx)


def weight(pb, alpha=None) -> np.ndarray:
    a = pb.alpha if alpha is None else alpha
    return (1.0 - a) * labeled_selector(pb) + a * laplacian(pb)


def centred_labels(pb) -> np.ndarray:
    y = np.zeros(pb.n)
    yl = np.where(np.asarray(pb.lab_y) > 0, 1.0, -1.0)
    y[pb.lab_idx] = yl - yl.mean()
    return y


def operator(pb, beta: float, alpha=None) -> np.ndarray:
    """A(beta) = (C X)^T M X + beta I (the one-sided form of Alg. 7)."""
    X = dense_x(pb)
    return (centring(pb) @ X).T @ weight(pb, alpha) @ X + beta * np.eye(pb.d)


def rhs(pb, r=None) -> np.ndarray:
    """Canonical (C X)^T y_c, or (C X)^T W_full X r for a start vector r."""
    X = dense_x(pb)
    B = centring(pb) @ X
    if r is None:
        return B.T @ centred_labels(pb)
    return B.T @ between_class_weight(pb) @ X @ r


def solve_dense(pb, beta: float, b=None, alpha=None) -> np.ndarray:
    if b is None:
        b = rhs(pb)
    return np.linalg.solve(operator(pb, beta, alpha), b)


def solve_pushthrough(pb, beta: float, alpha=None) -> np.ndarray:
    """w = B^T (M X B^T + beta I_N)^{-1} y_c with B = C X (canonical right-hand side)."""
    X = dense_x(pb)
    B = centring(pb) @ X
    K = weight(pb, alpha) @ X @ B.T + beta * np.eye(pb.n)
    return B.T @ np.linalg.solve(K, centred_labels(pb))


def solve_dual_ridge_alpha0(pb, beta: float) -> np.ndarray:
    """alpha = 0: ridge regression of the centred labels on the centred labeled rows."""
    X = dense_x(pb)
    Xl = X[pb.lab_idx]
    Xlc = Xl - Xl.mean(axis=0, keepdims=True)
    yl = np.where(np.asarray(pb.lab_y) > 0, 1.0, -1.0)
    yc = yl - yl.mean()
    G = Xlc @ Xlc.T + beta * np.eye(Xl.shape[0])
    return Xlc.T @ np.linalg.solve(G, yc)


# ---- spectral analysis for SDA (Alg. sasda), sample space ------------------

def sa_operator(pb, beta: float, alpha=None) -> np.ndarray:
    """C^T M I_N + beta I_N, C = I_N - 1 1_l^T / l (Alg. sasda, step 4)."""
    return centring(pb).T @ weight(pb, alpha) + beta * np.eye(pb.n)


def sa_rhs(pb, r=None) -> np.ndarray:
    """Canonical y_c, or W_full (r - 1 <1_l, r> / l) for a start vector r (Alg. sasda, steps 2-4)."""
    if r is None:
        return centred_labels(pb)
    ones_l = np.zeros(pb.n)
    ones_l[pb.lab_idx] = 1.0
    rr = np.asarray(r, dtype=np.float64) - np.ones(pb.n) * (ones_l @ r) / len(pb.lab_idx)
    return between_class_weight(pb) @ rr


def sa_solve_dense(pb, beta: float, g=None, alpha=None) -> np.ndarray:
    return np.linalg.solve(sa_operator(pb, beta, alpha), sa_rhs(pb) if g is None else g)


# ---- regression phase (Alg. optimizedSR, step 5) ---------------------------

def reg_solve_dense(pb, beta: float, z) -> np.ndarray:
    """LU of X^T X + beta I against X^T z."""
    X = dense_x(pb)
    return np.linalg.solve(X.T @ X + beta * np.eye(pb.d), X.T @ z)


def reg_solve_svd(pb, beta: float, z) -> np.ndarray:
    """Through the thin SVD X = U diag(s) V^T: w = V diag(s / (s^2 + beta)) U^T z."""
    U, sv, Vt = np.linalg.svd(dense_x(pb), full_matrices=False)
    return Vt.T @ ((sv / (sv * sv + beta)) * (U.T @ z))
