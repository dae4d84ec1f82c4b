"""Batched targets (fsda_multishift_solve_batch) vs the CPU oracle, one oracle solve per target.

Each target is the SDA problem of the shared X and S with its own labeled set;
the bar is the FP64 one, a relative solution error of 1e-6 per (target, shift).
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


def check_against_oracle(pb, labs, W, relres, betas, alpha, rtol):
    W = W.cpu().numpy()
    for c, (idx, y) in enumerate(labs):
        pc = dataclasses.replace(pb, lab_idx=idx, lab_y=y)
        Wr, *_ = oracle.solve(pc, betas=betas, rtol=1e-13, maxit=50000, alpha=alpha)
        for s in range(len(betas)):
            assert relerr(W[c, s], Wr[s]) < 1e-6, (c, s, relerr(W[c, s], Wr[s]))
            assert relres[c, s] < 20 * rtol, (c, s, relres[c, s])


@pytest.mark.parametrize("alpha", [1.0, 0.5, 0.0])
def test_batch_targets_match_oracle(tiny, alpha):
    labs = synth.target_labels(tiny, 5, seed=3, frac_median=0.05, frac_hi=0.2)
    op = fsda.Operator.from_problem(tiny, alpha=alpha)
    W, iters, relres, st = op.solve_batch(labs, tiny.betas, rtol=1e-10)
    assert st == fsda.OK
    check_against_oracle(tiny, labs, W, relres, tiny.betas, alpha, 1e-10)
    # the seed (smallest beta) stops last within each target
    assert np.all(iters.max(axis=1) == iters[:, np.argmin(tiny.betas)])


@pytest.mark.parametrize("ntarget", [1, 6, 9, 20, 37])
def test_batch_every_tile(tiny, ntarget):
    """1, 6 and 9 targets run with 4, 8 and 16 columns (padding included); 20 and 37
    in tiles of 16 (16 + 4; 16 + 16 + 5), one after the other."""
    labs = synth.target_labels(tiny, ntarget, seed=ntarget, frac_median=0.03, frac_hi=0.1)
    betas = np.array([3e-2, 0.4, 7.0])
    op = fsda.Operator.from_problem(tiny, alpha=0.5)
    W, iters, relres, st = op.solve_batch(labs, betas, rtol=1e-10, chunk=8)
    assert st == fsda.OK
    check_against_oracle(tiny, labs, W, relres, betas, 0.5, 1e-10)


def test_batch_equals_single_target_path(tiny):
    """A target of the batch and the single-target solve of the same labeled set agree."""
    labs = synth.target_labels(tiny, 3, seed=11, frac_median=0.05, frac_hi=0.2)
    op = fsda.Operator.from_problem(tiny, alpha=0.5)
    W, iters, relres, st = op.solve_batch(labs, tiny.betas, rtol=1e-11)
    for c, (idx, y) in enumerate(labs):
        single = fsda.Operator.from_problem(dataclasses.replace(tiny, lab_idx=idx, lab_y=y), alpha=0.5)
        Ws, its, rs, _ = single.solve(tiny.betas, rtol=1e-11)
        for s in range(tiny.betas.size):
            assert relerr(W[c, s].cpu().numpy(), Ws[s].cpu().numpy()) < 1e-7
        # the same recurrence with other summation orders: near rtol = 1e-11 the step at
        # which a shift crosses the threshold moves by a few iterations
        assert np.all(np.abs(iters[c] - its) <= np.maximum(2, 0.02 * its)), (iters[c], its)


def test_batch_label_order_and_determinism(tiny):
    labs = synth.target_labels(tiny, 4, seed=5, frac_median=0.05, frac_hi=0.2)
    rng = np.random.default_rng(0)
    shuffled = []
    for idx, y in labs:
        p = rng.permutation(idx.size)
        shuffled.append((idx[p], y[p]))
    op = fsda.Operator.from_problem(tiny)
    W1, it1, r1, _ = op.solve_batch(labs, tiny.betas, rtol=1e-9)
    W2, it2, r2, _ = op.solve_batch(shuffled, tiny.betas, rtol=1e-9)
    W3, it3, r3, _ = op.solve_batch(labs, tiny.betas, rtol=1e-9)
    assert torch.equal(W1, W2) and torch.equal(W1, W3)
    assert np.array_equal(it1, it2) and np.array_equal(r1, r3)


def test_batch_graph_equals_direct(tiny, monkeypatch):
    labs = synth.target_labels(tiny, 3, seed=7, frac_median=0.05, frac_hi=0.2)
    op_g = fsda.Operator.from_problem(tiny, alpha=0.5)
    monkeypatch.setenv("FSDA_NO_GRAPH", "1")
    op_d = fsda.Operator.from_problem(tiny, alpha=0.5)
    monkeypatch.delenv("FSDA_NO_GRAPH")
    for _ in range(2):
        Wg, itg, rg, _ = op_g.solve_batch(labs, tiny.betas, rtol=1e-9, chunk=16)
        Wd, itd, rd, _ = op_d.solve_batch(labs, tiny.betas, rtol=1e-9, chunk=16)
        torch.cuda.synchronize()
        assert torch.equal(Wg, Wd)
        assert np.array_equal(itg, itd)


def test_batch_ragged_problem():
    pb = synth.small_problem(n=77, d=4099, mean_nnz=3, k=2, alpha=0.7, seed=2, betas=(1e-3, 0.05, 2.0, 40.0),
                             n_lab=20)
    labs = synth.target_labels(pb, 3, seed=1, frac_median=0.3, frac_lo=0.1, frac_hi=0.5, pos_lo=0.3, pos_hi=0.6)
    op = fsda.Operator.from_problem(pb)
    W, iters, relres, st = op.solve_batch(labs, pb.betas, rtol=1e-11)
    assert st == fsda.OK
    check_against_oracle(pb, labs, W, relres, pb.betas, pb.alpha, 1e-11)


def test_batch_maxit_and_bad_labels(tiny):
    labs = synth.target_labels(tiny, 3, seed=9, frac_median=0.05, frac_hi=0.2)
    op = fsda.Operator.from_problem(tiny)
    W, iters, relres, st = op.solve_batch(labs, tiny.betas, rtol=1e-12, maxit=6, chunk=4)
    assert st == fsda.NOT_CONVERGED
    assert iters.max() == 6
    idx, y = labs[1]
    bad = list(labs)
    bad[1] = (np.concatenate([idx, idx[:1]]), np.concatenate([y, y[:1]]))
    with pytest.raises(fsda.FsdaError) as e:
        op.solve_batch(bad, tiny.betas, rtol=1e-8)
    assert e.value.code == fsda.E_LABELS and "target 1" in str(e.value)
    bad[1] = (idx, np.ones_like(y))
    with pytest.raises(fsda.FsdaError) as e:
        op.solve_batch(bad, tiny.betas, rtol=1e-8)
    assert e.value.code == fsda.E_LABELS


def test_batch_error_names_target_in_a_later_tile(tiny):
    """Targets past the first tile of 16 are named by their index in the call."""
    labs = synth.target_labels(tiny, 20, seed=13, frac_median=0.03, frac_hi=0.1)
    idx, y = labs[17]
    labs[17] = (idx, np.ones_like(y))
    op = fsda.Operator.from_problem(tiny)
    with pytest.raises(fsda.FsdaError) as e:
        op.solve_batch(labs, tiny.betas, rtol=1e-8)
    assert e.value.code == fsda.E_LABELS and "target 17" in str(e.value)


@pytest.mark.parametrize("tile", [4, 8])
def test_batch_set_tile_runs_smaller_tiles(tiny, tile):
    """A batch of 11 targets in tiles of 4 (4 + 4 + 3) or 8 (8 + 3) matches the oracle."""
    labs = synth.target_labels(tiny, 11, seed=21, frac_median=0.03, frac_hi=0.1)
    betas = np.array([5e-2, 1.0, 9.0])
    op = fsda.Operator.from_problem(tiny, alpha=0.5)
    op.set_batch_tile(tile)
    assert op.batch_tile == tile
    W, iters, relres, st = op.solve_batch(labs, betas, rtol=1e-10, chunk=8)
    assert st == fsda.OK
    check_against_oracle(tiny, labs, W, relres, betas, 0.5, 1e-10)
    with pytest.raises(fsda.FsdaError):
        op.set_batch_tile(12)
    assert op.batch_tile == tile
    op.set_batch_tile(0)
    assert op.batch_tile == 16


def test_batch_autotune_picks_a_shape_and_the_batch_stays_exact(tiny):
    """The tuner times tiles 4, 8 and 16 (9 targets allow all three) with 1, 2 and 4 groups
    of lanes per row, keeps the fastest shape, and the batch solved with it matches the oracle."""
    labs = synth.target_labels(tiny, 9, seed=8, frac_median=0.03, frac_hi=0.1)
    op = fsda.Operator.from_problem(tiny, alpha=0.5)
    tile, groups, rates = op.autotune_batch(labs, tiny.betas, trial_iters=16)
    assert (tile, groups) in rates
    assert set(rates) == {(t, g) for t in (4, 8, 16) for g in (1, 2, 4)} and all(r > 0 for r in rates.values())
    assert rates[(tile, groups)] == max(rates.values())
    assert (op.batch_tile, op.batch_groups) == (tile, groups)
    W, iters, relres, st = op.solve_batch(labs, tiny.betas, rtol=1e-10)
    assert st == fsda.OK
    check_against_oracle(tiny, labs, W, relres, tiny.betas, 0.5, 1e-10)
    # two targets: only the tile of 4 fits them
    tile2, groups2, rates2 = op.autotune_batch(labs[:2], tiny.betas, trial_iters=8)
    assert tile2 == 4 and {t for t, _ in rates2} == {4}


@pytest.mark.parametrize("tile,groups", [(4, 4), (8, 2), (16, 2), (16, 4)])
def test_batch_groups_per_row_match_oracle(tiny, tile, groups):
    """Rows of the row products shared by 2 or 4 groups of tile lanes (the X product with
    its mask features, the graph product, the short rows of X^T), ragged tiles included."""
    labs = synth.target_labels(tiny, 11, seed=tile + groups, frac_median=0.03, frac_hi=0.1)
    betas = np.array([3e-2, 0.4, 7.0])
    op = fsda.Operator.from_problem(tiny, alpha=0.5)
    op.set_batch_tile(tile)
    op.set_batch_groups(groups)
    W, iters, relres, st = op.solve_batch(labs, betas, rtol=1e-10, chunk=8)
    assert st == fsda.OK
    check_against_oracle(tiny, labs, W, relres, betas, 0.5, 1e-10)
    with pytest.raises(fsda.FsdaError):
        op.set_batch_groups(3)
    op.set_batch_groups(0)
    assert op.batch_groups == 1
