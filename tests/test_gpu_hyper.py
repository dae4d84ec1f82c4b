"""Hypergradients on the GPU: multi-column solve, hold-out loss, adjoint gradient, autograd wrapper."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from oracle import hyper as ohyper

torch = pytest.importorskip("torch")
fsda = pytest.importorskip("paper_1709_04794_amd")
from paper_1709_04794_amd import hyper  # noqa: E402

pytestmark = pytest.mark.gpu


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def tiny():
    return synth.workload("tiny")


def holdout_split(pb, seed=0, frac=0.2):
    rng = np.random.default_rng(seed)
    unl = np.setdiff1d(np.arange(pb.n), pb.lab_idx)
    ho = np.sort(rng.choice(unl, size=int(frac * unl.size), replace=False)).astype(np.int32)
    y = np.where(rng.random(ho.size) < 0.2, 1.0, -1.0)
    return ho, y


@pytest.mark.parametrize("ncol", [1, 5, 12])
def test_solve_columns_matches_oracle(tiny, ncol):
    op = fsda.Operator.from_problem(tiny, alpha=0.5)
    B = np.stack([oracle.rhs(tiny) * (1 + c) + synth.normal(tiny.d, seed=c, stream=4) for c in range(ncol)])
    sig = np.logspace(-2, 1, ncol)
    X, iters, relres, st = op.solve_columns(torch.from_numpy(B).cuda(), sig, rtol=1e-11)
    assert st == fsda.OK
    for c in range(ncol):
        ref = oracle.solve(tiny, betas=[sig[c]], rtol=1e-13, maxit=50000, b=B[c], alpha=0.5)[0][0]
        assert relerr(X[c].cpu().numpy(), ref) < 1e-6, c
        assert relres[c] < 20 * 1e-11


@pytest.mark.parametrize("alpha", [0.5, 1.0])
def test_loss_and_hypergradient_match_oracle(tiny, alpha):
    ho, y = holdout_split(tiny)
    betas = np.array([0.05, 0.6, 8.0])
    op = fsda.Operator.from_problem(tiny, alpha=alpha)
    W, *_ = op.solve(betas, rtol=1e-12)
    hi, hy = torch.from_numpy(ho).cuda(), torch.from_numpy(y).cuda()
    loss, G = op.holdout(W, hi, hy)
    Wn = W.cpu().numpy()
    assert np.allclose(loss, ohyper.loss(tiny, Wn, ho, y), rtol=1e-12, atol=0)
    Gr = ohyper.adjoint_rhs(tiny, Wn, ho, y)
    assert np.abs(G.cpu().numpy() - Gr).max() < 1e-12 * np.abs(Gr).max()
    Lam, it, rr, st = op.solve_columns(G, betas, rtol=1e-12)
    dlb, da = op.hypergradient(W, Lam, betas)
    H, dlb_r, da_r, _, _ = ohyper.gradients(tiny, betas, ho, y, alpha=alpha)
    assert np.allclose(loss, H, rtol=1e-8)
    assert np.allclose(dlb, dlb_r, rtol=1e-6, atol=1e-12 * np.abs(dlb_r).max()), (dlb, dlb_r)
    assert np.allclose(da, da_r, rtol=1e-6, atol=1e-12 * np.abs(da_r).max()), (da, da_r)


def test_holdout_rejects_bad_indices(tiny):
    op = fsda.Operator.from_problem(tiny)
    W, *_ = op.solve([1.0], rtol=1e-6)
    y = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(fsda.FsdaError):
        op.holdout(W, torch.tensor([3, tiny.n], dtype=torch.int32, device="cuda"), y)
    with pytest.raises(fsda.FsdaError):
        op.holdout(W, torch.tensor([3, 3], dtype=torch.int32, device="cuda"), y)


def test_autograd_matches_central_differences(tiny):
    ho, y = holdout_split(tiny, seed=2)
    obj = hyper.Objective(tiny, ho, y, rtol=1e-12)
    log_beta = torch.tensor(np.log([0.1, 2.0]), dtype=torch.float64, requires_grad=True)
    alpha = torch.tensor(0.6, dtype=torch.float64, requires_grad=True)
    H = hyper.HoldoutLoss.apply(log_beta, alpha, obj)
    H.sum().backward()
    h = 1e-4

    def f(lb, a):
        return hyper.HoldoutLoss.apply(torch.tensor(lb, dtype=torch.float64), torch.tensor(a, dtype=torch.float64),
                                       obj).detach().numpy()

    lb0 = log_beta.detach().numpy()
    for s in range(2):
        e = np.zeros(2)
        e[s] = h
        fd = (f(lb0 + e, 0.6)[s] - f(lb0 - e, 0.6)[s]) / (2 * h)
        assert abs(log_beta.grad[s].item() - fd) < 1e-5 * abs(fd), (s, log_beta.grad[s].item(), fd)
    fd_a = (f(lb0, 0.6 + h).sum() - f(lb0, 0.6 - h).sum()) / (2 * h)
    assert abs(alpha.grad.item() - fd_a) < 1e-5 * abs(fd_a), (alpha.grad.item(), fd_a)
