"""The target batch's shift-state fold on the matrix cores vs the vector-ALU fold
and the CPU oracle.

The fold adds, for every (target, shift), the chunk's buffered residuals with
their recurrence coefficients: a small dense product per target (16 shifts x
cnt residuals times cnt x columns), which ts_fold_apply_mfma runs with the FP64
16x16x4 matrix instruction, 4 residuals per step; FSDA_FOLD_MFMA=0 selects the
vector-ALU kernel.  The cases cover more than one group of 16 shifts (20 and 37
shifts), fold intervals that are not multiples of 4 (10, 13) beside the default,
and ragged tiles; both kernels are held to the oracle's FP64 bar (1e-6 per
solution) and to each other (they differ only in the order of the additions).
"""
import dataclasses

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


@pytest.mark.parametrize("nshift,chunk,ntarget", [(20, 10, 3), (37, 13, 5), (16, 0, 2)])
def test_fold_mfma_matches_valu_and_oracle(tiny, monkeypatch, nshift, chunk, ntarget):
    labs = synth.target_labels(tiny, ntarget, seed=nshift + 7, frac_median=0.05, frac_hi=0.2)
    betas = np.logspace(-2, 1.5, nshift)
    out = {}
    for mode in (None, "0"):
        if mode is None:
            monkeypatch.delenv("FSDA_FOLD_MFMA", raising=False)
        else:
            monkeypatch.setenv("FSDA_FOLD_MFMA", mode)
        op = fsda.Operator.from_problem(tiny, alpha=0.5, max_shifts=64)
        W, iters, relres, st = op.solve_batch(labs, betas, rtol=1e-10, chunk=chunk)
        assert st == fsda.OK
        assert (relres <= 20 * 1e-10).all(), (mode, relres.max())
        out[mode] = W.cpu().numpy()
        op.close()
    for c, (idx, y) in enumerate(labs):
        pc = dataclasses.replace(tiny, lab_idx=idx, lab_y=y)
        Wr, *_ = oracle.solve(pc, betas=betas, rtol=1e-13, maxit=50000, alpha=0.5)
        for s in range(nshift):
            for mode in (None, "0"):
                assert relerr(out[mode][c, s], Wr[s]) < 1e-6, (mode, c, s, relerr(out[mode][c, s], Wr[s]))
    assert relerr(out[None], out["0"]) < 1e-9
