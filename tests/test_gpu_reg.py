"""Regression-phase solve (fsda_regression_solve) vs the CPU oracle's per-shift CG.

Both the shared-basis recurrence and the independent per-shift CG baseline of
Table tab:shifted are checked against (X^T X + beta I) w = X^T z.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
fsda = pytest.importorskip("paper_1709_04794_amd")

pytestmark = pytest.mark.gpu


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def tiny():
    return synth.workload("tiny")


@pytest.mark.parametrize("shared", [True, False])
def test_regression_matches_oracle(tiny, shared):
    z = synth.normal(tiny.n, seed=3, stream=8)
    betas = np.logspace(-2, 2, 6)
    op = fsda.Operator.from_problem(tiny)
    W, iters, relres, st = op.regression_solve(torch.from_numpy(z).cuda(), betas, rtol=1e-10, shared_basis=shared)
    assert st == fsda.OK
    Wr, itr, *_ = oracle.reg_solve(tiny, z, betas, rtol=1e-13, maxit=50000)
    for s in range(betas.size):
        assert relerr(W[s].cpu().numpy(), Wr[s]) < 1e-6, (s, shared)
        assert relres[s] < 20 * 1e-10
    if shared:
        assert iters.max() == iters[np.argmin(betas)]


def test_shared_basis_and_per_shift_agree(tiny):
    """Each shift of the shared recurrence stops where its own CG would (same Krylov space)."""
    z = synth.normal(tiny.n, seed=5, stream=1)
    betas = np.array([1e-3, 1e-2, 0.1, 1.0, 10.0, 100.0])
    op = fsda.Operator.from_problem(tiny)
    zt = torch.from_numpy(z).cuda()
    Ws, its, rs, _ = op.regression_solve(zt, betas, rtol=1e-3, shared_basis=True)
    Wp, itp, rp, _ = op.regression_solve(zt, betas, rtol=1e-3, shared_basis=False)
    # the same iterates in exact arithmetic (Sec. 3.2.2); on this system the residual of
    # beta = 1e-2 stays within 3 % of rtol for iterations 94 to 96 (plain FP64 CG:
    # 1.03e-3, 0.92e-3, 0.83e-3), so the order of rounding moves its first crossing of
    # rtol by up to two iterations
    assert np.all(np.abs(its - itp) <= 2), (its, itp)
    for s in range(betas.size):
        # same iteration count: the same Krylov iterate in exact arithmetic; the two
        # recurrences (seeded at min beta and at beta_s) round differently, which the
        # conditioning amplifies over ~100 iterations (observed 1e-6 to 1.2e-5 here,
        # depending on the summation order of the dot products)
        bound = 1e-4 if its[s] == itp[s] else 1e-2
        assert relerr(Ws[s].cpu().numpy(), Wp[s].cpu().numpy()) < bound
        assert rs[s] <= 1.01e-3 and rp[s] <= 1.01e-3


def test_regression_ragged_chunks_and_repeat():
    pb = synth.small_problem(n=300, d=5000, mean_nnz=9, k=2, seed=2)
    z = synth.normal(pb.n, seed=1, stream=2)
    betas = np.array([1e-3, 0.05, 2.0, 40.0])
    op = fsda.Operator.from_problem(pb)
    zt = torch.from_numpy(z).cuda()
    ref, it0, _, _ = op.regression_solve(zt, betas, rtol=1e-11, chunk=32)
    W, it1, _, _ = op.regression_solve(zt, betas, rtol=1e-11, chunk=7)
    assert np.array_equal(it0, it1)  # the fold interval changes W only through its rounding
    assert relerr(W.cpu().numpy(), ref.cpu().numpy()) < 1e-12
    W2, _, _, _ = op.regression_solve(zt, betas, rtol=1e-11, chunk=7)
    assert torch.equal(W2, W)
    Wr, *_ = oracle.reg_solve(pb, z, betas, rtol=1e-13, maxit=50000)
    for s in range(betas.size):
        assert relerr(W[s].cpu().numpy(), Wr[s]) < 1e-6
