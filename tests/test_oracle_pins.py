"""Pins of the CPU oracle against facts the paper and the mathematics fix.

No GPU.  Each test checks the oracle (``oracle/fsda_oracle.c``) against
something other than itself: exact rational answers, dense solves through
different algebra, closed forms, special cases and invariants.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import dense, shifted

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "micro_exact.json")


def micro_problem(alpha):
    g = json.load(open(GOLDEN))
    rows = g["rows"]
    rp = np.zeros(len(rows) + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.concatenate([np.sort(r) for r in rows]).astype(np.int32)
    n = g["n"]
    adj = [set() for _ in range(n)]
    for i, j in g["edges"]:
        adj[i].add(j)
        adj[j].add(i)
    srp = np.zeros(n + 1, dtype=np.int32)
    srp[1:] = np.cumsum([len(a) for a in adj])
    scol = np.concatenate([sorted(a) for a in adj]).astype(np.int32)
    return synth.Problem(name="micro", n=n, d=g["d"], x_rowptr=rp, x_col=col, s_rowptr=srp, s_col=scol,
                         lab_idx=np.array(g["lab_idx"], dtype=np.int32),
                         lab_y=np.array(g["lab_y"], dtype=np.int8), alpha=float(alpha),
                         betas=np.array([1.0]), rtol=1e-14), g


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------------------
# exact rational golden values (tests/golden/micro_exact.json)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", range(9))
def test_golden_micro_exact(case):
    g = json.load(open(GOLDEN))
    c = g["cases"][case]
    pb, _ = micro_problem(float(Fraction(c["alpha"])))
    beta = float(Fraction(c["beta"]))
    b = oracle.rhs(pb)
    assert np.array_equal(b, np.array([float(Fraction(v)) for v in c["b"]]))
    W, it, rel, rc = oracle.solve(pb, betas=[beta], rtol=1e-15, maxit=200)
    assert relerr(W[0], np.array(c["w_float"])) < 1e-12


# ---------------------------------------------------------------------------
# dense solves through different algebra
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("alpha", [0.0, 0.3, 0.5, 1.0])
def test_oracle_vs_dense_lu(seed, alpha):
    pb = synth.small_problem(n=48, d=36, mean_nnz=5, k=3, alpha=alpha, seed=seed)
    W, it, rel, rc = oracle.solve(pb, rtol=1e-13, maxit=5000)
    assert rc == oracle.OK
    for s, beta in enumerate(pb.betas):
        ref = dense.solve_dense(pb, beta)
        assert relerr(W[s], ref) < 1e-9, (s, beta)
        assert rel[s] < 1e-12


@pytest.mark.parametrize("alpha", [0.2, 1.0])
def test_oracle_vs_pushthrough(alpha):
    pb = synth.small_problem(n=40, d=70, mean_nnz=6, k=4, alpha=alpha, seed=5)
    W, *_ = oracle.solve(pb, rtol=1e-13, maxit=5000)
    for s, beta in enumerate(pb.betas):
        assert relerr(W[s], dense.solve_pushthrough(pb, beta)) < 1e-9


def test_alpha0_is_ridge_on_centred_labeled_rows():
    pb = synth.small_problem(n=60, d=50, mean_nnz=6, k=3, n_lab=20, alpha=0.0, seed=7)
    W, *_ = oracle.solve(pb, rtol=1e-13, maxit=5000)
    for s, beta in enumerate(pb.betas):
        assert relerr(W[s], dense.solve_dual_ridge_alpha0(pb, beta)) < 1e-9


# ---------------------------------------------------------------------------
# special cases and invariants
# ---------------------------------------------------------------------------

def test_empty_graph_alpha1_gives_b_over_beta():
    pb = synth.small_problem(n=30, d=25, alpha=1.0, seed=3)
    pb.s_rowptr = np.zeros(pb.n + 1, dtype=np.int32)
    pb.s_col = np.zeros(0, dtype=np.int32)
    b = oracle.rhs(pb)
    W, it, rel, rc = oracle.solve(pb, rtol=1e-14, maxit=10)
    for s, beta in enumerate(pb.betas):
        assert np.allclose(W[s], b / beta, rtol=1e-15, atol=0)
        assert it[s] == 1


def test_ones_column_is_annihilated():
    """A feature present in every sample maps to X e_j = 1, which centring removes (Sec. 3.2.3)."""
    pb = synth.small_problem(n=30, d=20, alpha=0.4, seed=4)
    rows = [sorted(set(pb.x_col[pb.x_rowptr[i]:pb.x_rowptr[i + 1]].tolist()) | {0}) for i in range(pb.n)]
    pb.x_rowptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    pb.x_col = np.concatenate(rows).astype(np.int32)
    e0 = np.zeros(pb.d)
    e0[0] = 1.0
    beta = 0.7
    q = oracle.apply(pb, beta, e0)
    assert np.abs(q - beta * e0).max() < 1e-13
    W, *_ = oracle.solve(pb, rtol=1e-13, maxit=5000)
    assert np.abs(W[:, 0]).max() < 1e-12 * np.abs(W).max()


@pytest.mark.parametrize("alpha", [0.0, 0.25, 0.9])
def test_ones_vector_is_sa_eigenvector(alpha):
    """L 1 = 0, so 1 is an eigenvector of the SA problem with lambda_nd = 1/(1-alpha) (Sec. 2.5.2)."""
    pb = synth.small_problem(n=40, d=30, alpha=alpha, seed=8)
    ones = np.ones(pb.n)
    m1 = oracle.m_apply(pb, ones)
    w1 = dense.between_class_weight(pb) @ ones
    assert np.allclose(w1, m1 / (1.0 - alpha), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("alpha", [0.0, 0.5, 1.0])
def test_centring_annihilates_nondiscriminative_vector(alpha):
    """Xc^T [(1-alpha) P_l + alpha L] 1 = 0 (derivation in Sec. 3.2.3)."""
    pb = synth.small_problem(n=50, d=40, alpha=alpha, seed=9)
    v = oracle.xct(pb, oracle.m_apply(pb, np.ones(pb.n)))
    scale = oracle.xct(pb, np.ones(pb.n))
    assert np.abs(v).max() <= 1e-13 * max(1.0, np.abs(scale).max())


def test_operator_symmetric_and_two_sided_equals_one_sided():
    pb = synth.small_problem(n=50, d=40, alpha=0.35, seed=10)
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal(pb.d), rng.standard_normal(pb.d)
    Au, Av = oracle.apply(pb, 0.1, u), oracle.apply(pb, 0.1, v)
    assert abs(Au @ v - u @ Av) < 1e-12 * np.linalg.norm(Au) * np.linalg.norm(v)
    assert relerr(Au, dense.operator(pb, 0.1) @ u) < 1e-13


def test_rhs_closed_form_and_alg7_collinearity():
    """b = Xc^T y_c = (2 N+ N- / l)(mu+ - mu-); the Alg. 7 right-hand side is ((m+ - m-)/2) b."""
    pb = synth.small_problem(n=60, d=45, alpha=0.5, seed=11)
    X = dense.dense_x(pb)
    y = np.asarray(pb.lab_y)
    pos, neg = pb.lab_idx[y > 0], pb.lab_idx[y < 0]
    npos, nneg, l = pos.size, neg.size, pb.lab_idx.size
    b = oracle.rhs(pb)
    closed = 2.0 * npos * nneg / l * (X[pos].mean(0) - X[neg].mean(0))
    assert relerr(b, closed) < 1e-13
    r = synth.uniform(pb.d, -1.0, 1.0, seed=3, stream=5)
    b_lit = oracle.rhs(pb, r)
    xr = X @ r
    scale = (xr[pos].mean() - xr[neg].mean()) / 2.0
    assert relerr(b_lit, scale * b) < 1e-12
    assert relerr(b_lit, dense.rhs(pb, r)) < 1e-12


def test_large_shift_asymptotics():
    """w = b/beta - A0 b / beta^2 + O(beta^-3)."""
    pb = synth.small_problem(n=40, d=30, alpha=0.5, seed=12)
    b = oracle.rhs(pb)
    beta = 1e4
    W, *_ = oracle.solve(pb, betas=[beta], rtol=1e-15, maxit=100)
    a0b = oracle.apply(pb, 0.0, b)
    approx = b / beta - a0b / beta ** 2
    a0a0b = oracle.apply(pb, 0.0, a0b)
    bound = 2.0 * np.linalg.norm(a0a0b) / beta ** 3
    assert np.linalg.norm(W[0] - approx) <= bound + 1e-15 * np.linalg.norm(b / beta)


def test_sample_and_feature_permutation_invariance():
    pb = synth.small_problem(n=45, d=35, alpha=0.6, seed=13)
    W, *_ = oracle.solve(pb, rtol=1e-13, maxit=5000)
    rng = np.random.default_rng(1)
    ps = rng.permutation(pb.n)      # new row k is old row ps[k]
    pf = rng.permutation(pb.d)      # new feature pf[j] is old feature j
    inv_s = np.argsort(ps)
    X = dense.dense_x(pb)[ps][:, np.argsort(pf)]
    S = dense.dense_s(pb)[np.ix_(ps, ps)]
    q = synth.Problem(name="perm", n=pb.n, d=pb.d,
                      x_rowptr=np.concatenate([[0], np.cumsum(X.sum(1))]).astype(np.int32),
                      x_col=np.concatenate([np.nonzero(r)[0] for r in X]).astype(np.int32),
                      s_rowptr=np.concatenate([[0], np.cumsum(S.sum(1))]).astype(np.int32),
                      s_col=np.concatenate([np.nonzero(r)[0] for r in S]).astype(np.int32),
                      lab_idx=inv_s[pb.lab_idx].astype(np.int32), lab_y=pb.lab_y.copy(), alpha=pb.alpha,
                      betas=pb.betas, rtol=pb.rtol)
    Wq, *_ = oracle.solve(q, rtol=1e-13, maxit=5000)
    assert relerr(Wq[:, pf], W) < 1e-10


def test_projection_is_plain_xw():
    pb = synth.small_problem(n=40, d=30, alpha=0.5, seed=14)
    W, *_ = oracle.solve(pb, rtol=1e-12, maxit=5000)
    Sx = oracle.project(pb, W)
    assert np.allclose(Sx, W @ dense.dense_x(pb).T, rtol=1e-13, atol=1e-13)


def test_breakdown_is_reported_for_indefinite_weight():
    """alpha far outside [0, 1] makes the weight indefinite; CG must report breakdown."""
    pb = synth.small_problem(n=40, d=30, alpha=0.5, seed=15)
    b = oracle.rhs(pb)
    for alpha in (-2.0, -5.0, -20.0, -100.0):
        if b @ (dense.operator(pb, 1e-3, alpha=alpha) @ b) < 0:
            break
    else:
        pytest.skip("no indefinite alpha found")
    with pytest.raises(RuntimeError, match="status -5"):
        oracle.solve(pb, betas=[1e-3], alpha=alpha, rtol=1e-12, maxit=100)


# ---------------------------------------------------------------------------
# the reading of the shift recurrences (Alg. 3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("alpha", [0.5, 1.0])
def test_shifted_cg_matches_per_shift_cg(alpha):
    pb = synth.small_problem(n=60, d=80, mean_nnz=7, k=4, alpha=alpha, seed=16,
                             betas=(1e-2, 3e-2, 0.1, 1.0, 10.0, 100.0))
    b = oracle.rhs(pb)
    W_ref, *_ = oracle.solve(pb, rtol=1e-14, maxit=10000)
    s0 = pb.betas.min()
    tol = 1e-13 * np.linalg.norm(b)
    W, it, stop = shifted.shifted_cg(lambda p: oracle.apply(pb, s0, p), b, pb.betas - s0, tol, 5000)
    for s in range(pb.betas.size):
        assert relerr(W[s], W_ref[s]) < 1e-8, s
    # the printed index (alpha_i instead of alpha_{i+1}) breaks the collinearity
    Wp, *_ = shifted.shifted_cg(lambda p: oracle.apply(pb, s0, p), b, pb.betas - s0, tol, 5000, index="printed")
    assert max(relerr(Wp[s], W_ref[s]) for s in range(1, pb.betas.size)) > 1e-3


def test_lanczos_condition_matches_dense_spectrum():
    """kappa-hat from the CG coefficients (Sec. 3.2.1): run to convergence on a small
    problem, the Lanczos tridiagonal's extreme eigenvalues are the extreme
    eigenvalues of A(beta) over the eigenvectors b touches (dense eigh), for
    every shift, and every Ritz value lies inside A's spectrum."""
    pb = synth.small_problem(n=60, d=50, mean_nnz=6, k=3, alpha=0.5, seed=2)
    betas = np.array([0.01, 1.0, 30.0])
    kap, lo, hi, it = oracle.lanczos_condition(pb, betas=betas, rtol=1e-13, maxit=500)
    b = dense.rhs(pb)
    for s, beta in enumerate(betas):
        ev, V = np.linalg.eigh(dense.operator(pb, beta))
        touched = np.abs(V.T @ b) > 1e-10 * np.linalg.norm(b)
        # every Ritz value lies in the hull of the spectrum b touches
        assert ev[touched].min() * (1 - 1e-9) <= lo[s] and hi[s] <= ev[touched].max() * (1 + 1e-9), s
        if it[s] >= touched.sum():  # the run exhausted the Krylov space: the extremes are exact
            assert abs(hi[s] - ev[touched].max()) < 1e-8 * ev.max(), (s, hi[s], ev[touched].max())
            assert abs(lo[s] - ev[touched].min()) < 1e-6 * ev[touched].min(), (s, lo[s], ev[touched].min())
            assert abs(kap[s] - ev[touched].max() / ev[touched].min()) < 1e-5 * kap[s]
    assert it[0] >= 50 and it[1] >= 50  # the two small shifts exhaust it
    # shifting A shifts every Ritz value (the Krylov space does not depend on beta)
    assert abs((lo[1] - betas[1]) - (lo[0] - betas[0])) < 1e-6 * (lo[0] - betas[0])
