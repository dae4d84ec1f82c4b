"""Exact rational solve of the SDA system on micro problems -- TEST INFRASTRUCTURE ONLY.

Builds A(beta) = (X - 1 mu_l^T)^T [(1-alpha) P_l + alpha (D - S)] X + beta I and
the canonical right-hand side (X - 1 mu_l^T)^T y_c (Alg. 7, Sec. 2.3,
Sec. 3.2.3) with Python ``fractions.Fraction`` entries and solves it by
Gauss-Jordan elimination, so the answer carries no rounding at all.  Used to
write the golden fixture under ``tests/golden/``.
"""
from __future__ import annotations

from fractions import Fraction as F


def _matmul(A, B):
    n, k, m = len(A), len(B), len(B[0])
    return [[sum((A[i][t] * B[t][j] for t in range(k)), F(0)) for j in range(m)] for i in range(n)]


def _transpose(A):
    return [list(r) for r in zip(*A)]


def system(n, d, rows, edges, lab_idx, lab_y, alpha, beta):
    """rows: list of feature-id lists; edges: undirected (i, j) pairs, i != j."""
    X = [[F(0)] * d for _ in range(n)]
    for i, feats in enumerate(rows):
        for j in feats:
            X[i][j] = F(1)
    S = [[F(0)] * n for _ in range(n)]
    for i, j in edges:
        S[i][j] = F(1)
        S[j][i] = F(1)
    L = [[(sum(S[i]) if i == j else F(0)) - S[i][j] for j in range(n)] for i in range(n)]
    l = len(lab_idx)
    lab = [F(0)] * n
    for i in lab_idx:
        lab[i] = F(1)
    M = [[(1 - alpha) * (lab[i] if i == j else F(0)) + alpha * L[i][j] for j in range(n)] for i in range(n)]
    mu = [sum((lab[i] * X[i][j] for i in range(n)), F(0)) / l for j in range(d)]
    Xc = [[X[i][j] - mu[j] for j in range(d)] for i in range(n)]
    A = _matmul(_matmul(_transpose(Xc), M), X)
    for j in range(d):
        A[j][j] += beta
    ys = [F(1) if y > 0 else F(-1) for y in lab_y]
    ybar = sum(ys, F(0)) / l
    yc = [F(0)] * n
    for i, y in zip(lab_idx, ys):
        yc[i] = y - ybar
    b = [sum((Xc[i][j] * yc[i] for i in range(n)), F(0)) for j in range(d)]
    return A, b


def solve(A, b):
    """Gauss-Jordan elimination in exact arithmetic (A nonsingular)."""
    m = len(b)
    T = [list(A[i]) + [b[i]] for i in range(m)]
    for c in range(m):
        piv = next(r for r in range(c, m) if T[r][c] != 0)
        T[c], T[piv] = T[piv], T[c]
        pv = T[c][c]
        T[c] = [v / pv for v in T[c]]
        for r in range(m):
            if r != c and T[r][c] != 0:
                f = T[r][c]
                T[r] = [vr - f * vc for vr, vc in zip(T[r], T[c])]
    return [T[i][m] for i in range(m)]
