"""The paper's shifted conjugate gradient (Alg. 3) in NumPy -- TEST INFRASTRUCTURE ONLY.

Written in the paper's notation (gamma_i = -<r,r>/<p,q>, alpha_{i+1} the
direction coefficient, zeta the residual collinearity factors) to pin the
reading of its shift recurrences against independent per-shift solves:

  * the update of the per-shift direction coefficient is printed with alpha_i;
    the recurrence that keeps the shifted residuals collinear with the base
    residual needs the freshly computed alpha_{i+1} (as in Jegerlehner's
    multi-shift CG).  ``index="printed"`` keeps the printed form so a test can
    show it does not reproduce the per-shift solutions;
  * the base system is ``apply_base`` (any symmetric positive definite
    operator); each shift solves (base + sigma I) w = b;
  * a shift stops updating once |zeta| ||r|| <= tol.
"""
from __future__ import annotations

import numpy as np


def shifted_cg(apply_base, b: np.ndarray, sigmas, tol: float, maxit: int, index: str = "corrected"):
    """Returns (W [S, d], iterations of the base recurrence, per-shift stop iteration)."""
    sig = np.asarray(sigmas, dtype=np.float64)
    S = sig.size
    r = b.astype(np.float64).copy()
    p = r.copy()
    W = np.zeros((S, b.size))
    P = np.tile(r, (S, 1))
    alpha = 0.0            # alpha_0
    gamma_prev = 1.0       # gamma_{-1}
    zeta_prev = np.ones(S)  # zeta_{-1}
    zeta = np.ones(S)       # zeta_0
    active = np.ones(S, dtype=bool)
    stop_at = np.full(S, -1)
    rr = float(r @ r)
    it = 0
    for i in range(maxit):
        q = apply_base(p)
        gamma = -rr / float(p @ q)
        a = active
        zeta_next = zeta.copy()
        zeta_next[a] = (zeta_prev[a] * zeta[a] * gamma_prev /
                        (gamma * alpha * (zeta_prev[a] - zeta[a]) +
                         zeta_prev[a] * gamma_prev * (1.0 - sig[a] * gamma)))
        gamma_s = np.zeros(S)
        gamma_s[a] = gamma * zeta_next[a] / zeta[a]
        W[a] -= gamma_s[a, None] * P[a]
        r = r + gamma * q
        it = i + 1
        rr_next = float(r @ r)
        rnorm = np.sqrt(rr_next)
        if rnorm < tol:
            stop_at[active] = it
            break
        alpha_next = rr_next / rr
        p = r + alpha_next * p
        coef = alpha_next if index == "corrected" else alpha
        alpha_s = np.zeros(S)
        alpha_s[a] = coef * zeta_next[a] * gamma_s[a] / (zeta[a] * gamma)
        P[a] = zeta_next[a, None] * r[None, :] + alpha_s[a, None] * P[a]
        done = a & (np.abs(zeta_next) * rnorm < tol)
        stop_at[done] = it
        active = a & ~done
        zeta_prev, zeta = zeta, zeta_next
        gamma_prev, alpha, rr = gamma, alpha_next, rr_next
        if not active.any():
            break
    return W, it, stop_at
