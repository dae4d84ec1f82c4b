"""LDS slices of the batched X^T product (targets, per-target columns, multi-column
solves) vs the CPU oracle and vs the plan without them.

The longest rows of X^T (at least 16 nonzeros per slice on average, or the
threshold FSDA_BXT_LDS_SEG sets; 0 turns the slices off) are summed per slice
of 128 KiB / (8 T) samples from u staged in LDS, each segment's 16-bit offsets
padded to a multiple of 8 with a zero row; their parts are added in slice order.
The tiny workload (2,000 samples: two slices at T = 16, every chunked row taken)
and a planted problem (300,000 samples, 293 slices at T = 16: the five features
of >= 4,688 nonzeros taken, the others chunked and cut into XCD slices) run
with and without them; a threshold of 1 takes every chunked row, down to
segments of a single nonzero (mostly padding).  The multi-column solves run
tiles of 4, 16 and 64 columns (slices of 4096, 1024 and 256 samples).  The plans differ only in the
order of additions, so they agree to rounding; the oracle bars are the FP64 ones.
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


def build(pb, monkeypatch, seg, **kw):
    """seg: the LDS-slice threshold (None: the default; "0": off)."""
    if seg is None:
        monkeypatch.delenv("FSDA_BXT_LDS_SEG", raising=False)
    else:
        monkeypatch.setenv("FSDA_BXT_LDS_SEG", str(seg))
    monkeypatch.delenv("FSDA_BXT_SLICES", raising=False)
    monkeypatch.delenv("FSDA_BXT_SLICE_MIN", raising=False)
    return fsda.Operator.from_problem(pb, **kw)


@pytest.fixture(scope="module")
def tiny():
    return synth.workload("tiny")


@pytest.fixture(scope="module")
def planted():
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


@pytest.mark.parametrize("tile", [4, 8, 16])
def test_lds_targets_tiny_match_oracle_and_plain(tiny, monkeypatch, tile):
    labs = synth.target_labels(tiny, 6, seed=tile + 60, frac_median=0.05, frac_hi=0.2)
    betas = np.array([2e-2, 0.3, 5.0])
    out = {}
    for seg in (None, "0"):
        op = build(tiny, monkeypatch, seg, alpha=0.5)
        op.set_batch_tile(tile)
        W, iters, relres, st = op.solve_batch(labs, betas, rtol=1e-10, chunk=16)
        assert st == fsda.OK
        out[seg] = W.cpu().numpy()
        if seg is None:
            check_targets(tiny, labs, W, relres, betas, 0.5, 1e-10)
        op.close()
    assert relerr(out[None], out["0"]) < 1e-9


@pytest.mark.parametrize("seg", [None, "1"])
def test_lds_targets_planted_match_oracle(planted, monkeypatch, seg):
    labs = synth.target_labels(planted, 3, seed=9, frac_median=0.01, frac_hi=0.02)
    betas = np.array([0.05, 5.0])
    op = build(planted, monkeypatch, seg, alpha=0.5)
    W, iters, relres, st = op.solve_batch(labs, betas, rtol=1e-11)
    assert st == fsda.OK
    check_targets(planted, labs, W, relres, betas, 0.5, 1e-11)


def test_lds_columns_batch_planted(planted, monkeypatch):
    labs = synth.target_labels(planted, 2, seed=3, frac_median=0.01, frac_hi=0.02)
    betas = np.array([0.05, 5.0])
    B = np.stack([np.stack([synth.normal(planted.d, seed=10 * c + s, stream=6) for s in range(2)]) for c in range(2)])
    op = build(planted, monkeypatch, None, alpha=0.5)
    X, iters, relres, st = op.solve_columns_batch(labs, betas, torch.from_numpy(B).cuda(), rtol=1e-11)
    assert st == fsda.OK
    X = X.cpu().numpy()
    for c in range(2):
        pc = dataclasses.replace(planted, lab_idx=labs[c][0], lab_y=labs[c][1])
        for s in range(2):
            ref = oracle.solve(pc, betas=[betas[s]], rtol=1e-13, maxit=50000, b=B[c, s], alpha=0.5)[0][0]
            assert relerr(X[c, s], ref) < 1e-6, (c, s, relerr(X[c, s], ref))


@pytest.mark.parametrize("ncol", [3, 16, 40])
def test_lds_columns_tiny_match_oracle_and_plain(tiny, monkeypatch, ncol):
    B = np.stack([oracle.rhs(tiny) * (1 + c) + synth.normal(tiny.d, seed=70 + c, stream=4) for c in range(ncol)])
    sig = np.logspace(-2, 1, ncol)
    out = {}
    for seg in (None, "0"):
        op = build(tiny, monkeypatch, seg, alpha=0.5)
        X, iters, relres, st = op.solve_columns(torch.from_numpy(B).cuda(), sig, rtol=1e-11)
        assert st == fsda.OK
        out[seg] = X.cpu().numpy()
        op.close()
    for c in range(ncol):
        ref = oracle.solve(tiny, betas=[sig[c]], rtol=1e-13, maxit=50000, b=B[c], alpha=0.5)[0][0]
        assert relerr(out[None][c], ref) < 1e-6, c
    assert relerr(out[None], out["0"]) < 1e-9
