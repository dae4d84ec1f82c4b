"""XCD slices of the batched X^T product (targets, multi-column and per-target
column solves) vs the CPU oracle and vs the unsliced plan.

With XCD slices the long rows of X^T are cut at the sample boundaries x n / 8
and summed in pieces that never cross one, so that each XCD gathers from one
eighth of the sample-space vector for them.  They are chosen when that
vector over the tile's columns outgrows an XCD's L2 share; FSDA_BXT_SLICES=8
or 0 forces them on or off, which is how these tests run both plans on the same
inputs.  Only rows of at least two chunks are cut by default
(FSDA_BXT_SLICE_MIN sets the shortest row cut; the tiny workload's rows are cut
from 64 nonzeros here, so that every row of the chunked part is cut).  The two
plans differ only in the order in which a long row's pieces are added, so they
agree to rounding; the oracle bars are the FP64 ones.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
fsda = pytest.importorskip("paper_1709_04794_amd")

pytestmark = pytest.mark.gpu

PLANTED_COUNTS = [300000, 120000, 20000, 9000, 5000, 3000, 1500, 800, 600, 400, 300, 200, 100, 80, 64,
                  63, 40, 20, 10, 5, 2, 1, 0, 0]


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def build(pb, monkeypatch, slices, slice_min=None, **kw):
    """slices "8" or "0"; slice_min: the shortest row cut into slices (default: eight chunks).
    The LDS slices of the longest rows are off here (they would take every chunked row of
    the tiny workload; tests/test_gpu_bxt_lds.py covers them)."""
    monkeypatch.setenv("FSDA_BXT_LDS_SEG", "0")
    monkeypatch.setenv("FSDA_BXT_SLICES", str(slices))
    if slice_min is None:
        monkeypatch.delenv("FSDA_BXT_SLICE_MIN", raising=False)
    else:
        monkeypatch.setenv("FSDA_BXT_SLICE_MIN", str(slice_min))
    return fsda.Operator.from_problem(pb, **kw)


@pytest.fixture(scope="module")
def tiny():
    return synth.workload("tiny")


@pytest.fixture(scope="module")
def planted():
    """300,000 samples, 24 features of planted lengths: a dense feature (pieces of every
    slice longer than one chunk), rows of every length class, short and empty rows."""
    return synth.planted_problem(300000, PLANTED_COUNTS, n_lab=3000, pos_frac=0.3, alpha=0.5,
                                 betas=(0.05, 0.5, 5.0, 50.0), seed=4, rtol=1e-11)


def check_targets(pb, labs, W, relres, betas, alpha, rtol):
    W = W.cpu().numpy()
    for c, (idx, y) in enumerate(labs):
        pc = dataclasses.replace(pb, lab_idx=idx, lab_y=y)
        Wr, *_ = oracle.solve(pc, betas=betas, rtol=1e-13, maxit=50000, alpha=alpha)
        for s in range(len(betas)):
            assert relerr(W[c, s], Wr[s]) < 1e-6, (c, s, relerr(W[c, s], Wr[s]))
            assert relres[c, s] < 20 * rtol, (c, s, relres[c, s])


@pytest.mark.parametrize("ntarget", [5, 20])
def test_sliced_batch_targets_match_oracle_and_unsliced(tiny, monkeypatch, ntarget):
    labs = synth.target_labels(tiny, ntarget, seed=ntarget + 40, frac_median=0.05, frac_hi=0.2)
    betas = np.array([2e-2, 0.3, 5.0])
    out = {}
    for sl in ("8", "0"):
        op = build(tiny, monkeypatch, sl, slice_min=64, alpha=0.5)
        W, iters, relres, st = op.solve_batch(labs, betas, rtol=1e-10, chunk=16)
        assert st == fsda.OK
        out[sl] = W.cpu().numpy()
        if sl == "8":
            check_targets(tiny, labs, W, relres, betas, 0.5, 1e-10)
        op.close()
    assert relerr(out["8"], out["0"]) < 1e-9


@pytest.mark.parametrize("slice_min", [None, 64])
def test_sliced_batch_targets_planted(planted, monkeypatch, slice_min):
    """Default: the rows of >= 8192 nonzeros cut (pieces of 1024), the shorter ones in whole
    chunks after the sliced rounds; 64: every chunked row cut."""
    labs = synth.target_labels(planted, 3, seed=9, frac_median=0.01, frac_hi=0.02)
    betas = np.array([0.05, 5.0])
    op = build(planted, monkeypatch, "8", slice_min=slice_min, alpha=0.5)
    W, iters, relres, st = op.solve_batch(labs, betas, rtol=1e-11)
    assert st == fsda.OK
    check_targets(planted, labs, W, relres, betas, 0.5, 1e-11)


@pytest.mark.parametrize("ncol", [3, 16])
def test_sliced_columns_match_oracle(tiny, monkeypatch, ncol):
    B = np.stack([oracle.rhs(tiny) * (1 + c) + synth.normal(tiny.d, seed=50 + c, stream=4) for c in range(ncol)])
    sig = np.logspace(-2, 1, ncol)
    out = {}
    for sl in ("8", "0"):
        op = build(tiny, monkeypatch, sl, slice_min=64, alpha=0.5)
        X, iters, relres, st = op.solve_columns(torch.from_numpy(B).cuda(), sig, rtol=1e-11)
        assert st == fsda.OK
        out[sl] = X.cpu().numpy()
        op.close()
    for c in range(ncol):
        ref = oracle.solve(tiny, betas=[sig[c]], rtol=1e-13, maxit=50000, b=B[c], alpha=0.5)[0][0]
        assert relerr(out["8"][c], ref) < 1e-6, c
    assert relerr(out["8"], out["0"]) < 1e-9


def test_sliced_columns_batch_planted(planted, monkeypatch):
    labs = synth.target_labels(planted, 2, seed=3, frac_median=0.01, frac_hi=0.02)
    betas = np.array([0.05, 5.0])
    B = np.stack([np.stack([synth.normal(planted.d, seed=10 * c + s, stream=5) for s in range(2)]) for c in range(2)])
    op = build(planted, monkeypatch, "8", alpha=0.5)
    X, iters, relres, st = op.solve_columns_batch(labs, betas, torch.from_numpy(B).cuda(), rtol=1e-11)
    assert st == fsda.OK
    X = X.cpu().numpy()
    for c in range(2):
        pc = dataclasses.replace(planted, lab_idx=labs[c][0], lab_y=labs[c][1])
        for s in range(2):
            ref = oracle.solve(pc, betas=[betas[s]], rtol=1e-13, maxit=50000, b=B[c, s], alpha=0.5)[0][0]
            assert relerr(X[c, s], ref) < 1e-6, (c, s, relerr(X[c, s], ref))
