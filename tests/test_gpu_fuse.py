"""The residual update of the batched solves with and without its fusion into the
X^T product, vs the CPU oracle.

By default the batched X^T product does the CG update itself: in the target
batch r_{i+1} = r_i - a_c q into the residual ring, in the column solves (one
labeled set, per-target labeled sets, the mixed path's FP32 correction solves)
r = r - a_c q and x = x + a_c p on the interleaved vectors, with the partial
sums of <r, r> from the blocks of both of its levels (rows summed by one group,
rows summed in pieces).  FSDA_BXT_FUSE=0 keeps q and runs the separate update
kernel.  The two differ only in the order in which the partial sums are added,
so they agree to rounding; each is held to the oracle's FP64 bars (1e-6 per
solution, 1e-4 for the mixed path).  The tiny workload has X^T rows on both
sides of the 512-nonzero boundary, so both levels' epilogues run.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
fsda = pytest.importorskip("paper_1709_04794_amd")

pytestmark = pytest.mark.gpu

MODES = (None, "0")  # fused (the default), separate update kernel


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def build(pb, monkeypatch, fuse, **kw):
    if fuse is None:
        monkeypatch.delenv("FSDA_BXT_FUSE", raising=False)
    else:
        monkeypatch.setenv("FSDA_BXT_FUSE", fuse)
    return fsda.Operator.from_problem(pb, **kw)


@pytest.fixture(scope="module")
def tiny():
    return synth.workload("tiny")


def test_tiny_has_rows_on_both_sides_of_the_boundary(tiny):
    counts = np.bincount(np.asarray(tiny.x_col), minlength=tiny.d)
    assert (counts >= 512).sum() >= 1 and (counts < 512).sum() >= 1


@pytest.mark.parametrize("ncol", [3, 16, 40])
def test_columns_fused_and_separate_match_oracle(tiny, monkeypatch, ncol):
    B = np.stack([oracle.rhs(tiny) * (1 + c) + synth.normal(tiny.d, seed=90 + c, stream=4) for c in range(ncol)])
    sig = np.logspace(-2, 1, ncol)
    out = {}
    for fuse in MODES:
        op = build(tiny, monkeypatch, fuse, alpha=0.5)
        X, iters, relres, st = op.solve_columns(torch.from_numpy(B).cuda(), sig, rtol=1e-11)
        assert st == fsda.OK
        assert (relres <= 1e-11 * 20).all(), relres.max()
        out[fuse] = X.cpu().numpy()
        op.close()
    for c in range(ncol):
        ref = oracle.solve(tiny, betas=[sig[c]], rtol=1e-13, maxit=50000, b=B[c], alpha=0.5)[0][0]
        for fuse in MODES:
            assert relerr(out[fuse][c], ref) < 1e-6, (fuse, c, relerr(out[fuse][c], ref))
    assert relerr(out[None], out["0"]) < 1e-9


def test_columns_batch_per_target_fused_and_separate(tiny, monkeypatch):
    labs = synth.target_labels(tiny, 3, seed=31, frac_median=0.05, frac_hi=0.2)
    betas = np.array([2e-2, 0.4, 6.0])
    B = np.stack([np.stack([synth.normal(tiny.d, seed=10 * c + s, stream=7) for s in range(3)]) for c in range(3)])
    out = {}
    for fuse in MODES:
        op = build(tiny, monkeypatch, fuse, alpha=0.5)
        X, iters, relres, st = op.solve_columns_batch(labs, betas, torch.from_numpy(B).cuda(), rtol=1e-11)
        assert st == fsda.OK
        out[fuse] = X.cpu().numpy()
        op.close()
    for c in range(3):
        pc = dataclasses.replace(tiny, lab_idx=labs[c][0], lab_y=labs[c][1])
        for s in range(3):
            ref = oracle.solve(pc, betas=[betas[s]], rtol=1e-13, maxit=50000, b=B[c, s], alpha=0.5)[0][0]
            for fuse in MODES:
                assert relerr(out[fuse][c, s], ref) < 1e-6, (fuse, c, s)
    assert relerr(out[None], out["0"]) < 1e-9


@pytest.mark.parametrize("tile", [4, 16])
def test_targets_fused_and_separate(tiny, monkeypatch, tile):
    labs = synth.target_labels(tiny, 5, seed=tile + 40, frac_median=0.05, frac_hi=0.2)
    betas = np.array([2e-2, 0.3, 5.0])
    out = {}
    for fuse in MODES:
        op = build(tiny, monkeypatch, fuse, alpha=0.5)
        op.set_batch_tile(tile)
        W, iters, relres, st = op.solve_batch(labs, betas, rtol=1e-10, chunk=16)
        assert st == fsda.OK
        out[fuse] = W.cpu().numpy()
        op.close()
    for c, (idx, y) in enumerate(labs):
        pc = dataclasses.replace(tiny, lab_idx=idx, lab_y=y)
        Wr, *_ = oracle.solve(pc, betas=betas, rtol=1e-13, maxit=50000, alpha=0.5)
        for s in range(betas.size):
            for fuse in MODES:
                assert relerr(out[fuse][c, s], Wr[s]) < 1e-6, (fuse, c, s)
    assert relerr(out[None], out["0"]) < 1e-9


def test_mixed_correction_fused_and_separate(tiny, monkeypatch):
    betas = np.logspace(-2, 2, 5)
    Wr, *_ = oracle.solve(tiny, betas=betas, rtol=1e-13, maxit=20000, alpha=0.5)
    for fuse in MODES:
        op = build(tiny, monkeypatch, fuse, precision=fsda.MIXED, max_shifts=64, alpha=0.5)
        W, iters, relres, st = op.solve(betas, rtol=1e-9)
        assert st == fsda.OK
        assert (relres <= 1e-9).all(), (fuse, relres.max())
        W = W.cpu().numpy()
        for s in range(betas.size):
            assert relerr(W[s], Wr[s]) < 1e-4, (fuse, s, relerr(W[s], Wr[s]))
        op.close()
