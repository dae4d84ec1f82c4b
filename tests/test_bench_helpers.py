"""Host-side helpers of bench.py that build index streams and byte models: the
gather patterns are the products' own index sets, and the byte model adds up.
CPU only."""
import numpy as np
import pytest

import bench
import synth


def test_gather_patterns_are_the_products_index_sets():
    pb = synth.small_problem(n=120, d=3000, mean_nnz=20, k=3, seed=5)
    pat = bench.gather_patterns(pb)
    xt_rows, xt_cols, xt_size = pat["xt"]
    assert xt_size == pb.n and xt_cols.size == pb.x_col.size
    # the X^T stream lists, feature by feature (decreasing frequency), the samples of that feature
    cnt = np.bincount(pb.x_col, minlength=pb.d)
    assert np.all(np.diff(cnt[np.argsort(-cnt, kind="stable")][xt_rows]) <= 0)
    xrow = np.repeat(np.arange(pb.n), np.diff(pb.x_rowptr))
    assert sorted(zip(xt_cols.tolist(), xt_rows.tolist())) == sorted(
        zip(xrow.tolist(), np.argsort(np.argsort(-cnt, kind="stable"), kind="stable")[pb.x_col].tolist()))
    # the X stream beyond the features staged in shared memory
    xr, xc, xsize = pat["x_cold"]
    assert xsize == pb.d and np.all(xc >= bench.HOT_FEATURES)
    new = np.argsort(np.argsort(-cnt, kind="stable"), kind="stable")[pb.x_col]
    assert xc.size == int((new >= bench.HOT_FEATURES).sum())
    # the graph stream is S itself
    sr, sc, ssize = pat["s"]
    assert ssize == pb.n and np.array_equal(sc, pb.s_col)
    assert np.array_equal(sr, np.repeat(np.arange(pb.n), np.diff(pb.s_rowptr)))


@pytest.mark.parametrize("plan", ["1", "lds", "8"])
def test_operator_apply_bytes_are_the_sum_of_the_products(monkeypatch, plan):
    monkeypatch.setenv("FSDA_XT_SLICES", plan)
    pb = synth.small_problem(n=200, d=500, mean_nnz=30, k=3, seed=2)
    import paper_1709_04794_amd as fsda
    total = sum(bench.algorithmic_bytes(k, pb, 4, 32) for k in (fsda.K_X, fsda.K_S, fsda.K_XT, fsda.K_XTL,
                                                                 fsda.K_ASM))
    n, d, z, g = pb.n, pb.d, pb.x_nnz, pb.s_nnz
    lab = 16 * n if pb.alpha < 1.0 else 0
    # products as launched (the X^T pass also reads and writes r: 8d + 8d beyond the bare apply)
    want = 8 * z + 4 * g + 40 * n + 36 * d + 12 + lab
    pl = bench.xt_plan(pb)
    cnt = np.bincount(pb.x_col, minlength=d)
    split = cnt >= 64
    if plan == "lds":
        # two X^T kernels: u read by both, the split rows' slice bounds, parts written and read
        nsl, nsplit = pl["nsl"], pl["n_lds"]
        assert (pl["plan"], nsl) == ("lds", 1) and nsplit == int(split.sum()) > 0
        assert pl["z_lds"] == int(cnt[split].sum()) and pl["n_xcd"] == 0
        want += 8 * n + 4 * (nsl + 1) * nsplit + 16 * nsl * nsplit
    elif plan == "8":
        # the split rows' parts (8 per row, these rows are short) written by the X^T pass and read by
        # the assembly, which also reads their part offsets (p and r in, r out move with their rows)
        # (XCD slices take the rows of >= 16 nonzeros)
        assert pl["plan"] == "xcd" and pl["n_xcd"] == int((cnt >= 16).sum()) > int(split.sum()) > 0
        assert pl["n_lds"] == 0
        assert pl["xcd_parts"] == 8 * pl["n_xcd"]
        want += 16 * pl["xcd_parts"] + 4 * (pl["n_xcd"] + 1)
    else:
        assert pl["plan"] == "none"
    assert total == want


def test_xcd_sliced_stream_is_a_slice_aligned_permutation():
    """Same indices; piece p (256 entries, block p % grid, XCD p % 8) holds only slice
    p % 8; the non-aligned control spreads every slice over all eight positions."""
    pb = synth.workload("tiny")
    idx = bench.gather_patterns(pb)["xt"][1]
    n = pb.n
    for aligned in (True, False):
        s = bench.xcd_sliced_stream(idx, n, aligned=aligned)
        assert np.array_equal(np.sort(s), np.sort(idx))
        m = min(np.bincount((idx.astype(np.int64) * 8) // n, minlength=8)) // 256 * 256
        pieces = s[: 8 * m].reshape(-1, 256)
        sl = (pieces.astype(np.int64) * 8) // n
        assert (sl == sl[:, :1]).all()  # one slice per piece
        p = np.arange(len(pieces))
        if aligned:
            assert (sl[:, 0] == p % 8).all()
        else:
            assert (sl[:, 0] == (p % 8 + p // 8) % 8).all()
            assert len(np.unique(sl[p % 8 == 0, 0])) == min(8, len(pieces[p % 8 == 0]))


def test_every_function_bench_calls_is_defined():
    """Every bare name bench.py calls is bound somewhere in it (a function, an
    argument, an assignment) or is a builtin: a refactoring that drops a function
    still called by the default run fails here, on the CPU."""
    import ast
    import builtins
    tree = ast.parse(open(bench.__file__).read())
    bound = set()
    for node in ast.walk(tree):
        if isinstance(node, (ast.FunctionDef, ast.ClassDef)):
            bound.add(node.name)
        elif isinstance(node, ast.arg):
            bound.add(node.arg)
        elif isinstance(node, ast.Name) and isinstance(node.ctx, ast.Store):
            bound.add(node.id)
        elif isinstance(node, (ast.Import, ast.ImportFrom)):
            bound.update((a.asname or a.name).split(".")[0] for a in node.names)
    called = {n.func.id for n in ast.walk(tree) if isinstance(n, ast.Call) and isinstance(n.func, ast.Name)}
    missing = sorted(c for c in called if c not in bound and not hasattr(builtins, c))
    assert not missing, missing
    for name in ("batched_bench", "single_bench", "roofline_large", "diff_experiment", "cpu_baseline_targets"):
        assert callable(getattr(bench, name)), name
