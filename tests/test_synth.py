"""The seeded input generator: structure of X and of the Tanimoto kNN graph."""
import numpy as np
import pytest

import synth


def test_fingerprints_structure_and_determinism():
    rp, col = synth.fingerprints(500, 300, 12, 1.1, seed=4)
    assert rp[0] == 0 and rp[-1] == col.size
    lens = np.diff(rp)
    assert lens.min() >= 1
    for i in range(500):
        r = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(r) > 0)
        assert r.min() >= 0 and r.max() < 300
    rp2, col2 = synth.fingerprints(500, 300, 12, 1.1, seed=4)
    assert np.array_equal(rp, rp2) and np.array_equal(col, col2)
    rp3, col3 = synth.fingerprints(500, 300, 12, 1.1, seed=5)
    assert not np.array_equal(col, col3[:col.size]) or not np.array_equal(rp, rp3)
    # Zipf popularity: the most frequent feature is far above the mean
    cnt = np.bincount(col, minlength=300)
    assert cnt.max() > 10 * cnt.mean()


def _brute_knn(rows, k, ties):
    n = len(rows)
    sets = [set(r) for r in rows]
    nbr = []
    for i in range(n):
        sims = []
        for j in range(n):
            if j == i:
                continue
            inter = len(sets[i] & sets[j])
            un = len(sets[i] | sets[j])
            sims.append((inter / un if un else 0.0, j))
        sims.sort(key=lambda t: (-t[0], t[1]))
        keep = sims[:k]
        if ties:
            kth = keep[-1][0]
            keep = [t for t in sims if t[0] >= kth]
        nbr.append({j for _, j in keep})
    adj = [set() for _ in range(n)]
    for i in range(n):
        for j in nbr[i]:
            adj[i].add(j)
            adj[j].add(i)
    return adj


@pytest.mark.parametrize("ties", [True, False])
def test_knn_exact_matches_brute_force(ties):
    rp, col = synth.fingerprints(70, 40, 6, 1.1, seed=2)
    rows = [col[rp[i]:rp[i + 1]].tolist() for i in range(70)]
    srp, scol = synth.knn_graph(70, rp, col, 4, ties=ties, method="exact")
    ref = _brute_knn(rows, 4, ties)
    for i in range(70):
        assert set(scol[srp[i]:srp[i + 1]].tolist()) == ref[i]


def test_knn_graph_symmetric_no_self_loops():
    rp, col = synth.fingerprints(3000, 2000, 20, 1.1, seed=1)
    for method in ("exact", "lsh"):
        srp, scol = synth.knn_graph(3000, rp, col, 5, method=method)
        S = set()
        for i in range(3000):
            r = scol[srp[i]:srp[i + 1]]
            assert np.all(np.diff(r) > 0)
            assert i not in r
            assert r.size >= 1
            S.update((i, int(j)) for j in r)
        assert all((j, i) in S for (i, j) in S)


def test_labels_planted():
    rp, col = synth.fingerprints(1000, 500, 10, 1.1, seed=3)
    li, ly = synth.labels(1000, rp, col, 500, 100, 0.2, seed=3)
    assert li.size == 100 and np.all(np.diff(li) > 0)
    assert (ly > 0).sum() == 20 and (ly < 0).sum() == 80


def test_target_labels_are_valid_and_reproducible():
    pb = synth.workload("tiny")
    a = synth.target_labels(pb, 7, seed=4, frac_median=0.02)
    b = synth.target_labels(pb, 7, seed=4, frac_median=0.02)
    assert len(a) == 7
    for (i1, y1), (i2, y2) in zip(a, b):
        assert np.array_equal(i1, i2) and np.array_equal(y1, y2)
        assert i1.dtype == np.int32 and y1.dtype == np.int8
        assert np.unique(i1).size == i1.size and i1.min() >= 0 and i1.max() < pb.n
        assert set(np.unique(y1).tolist()) == {-1, 1}
        assert i1.size >= 4
    assert len({i.size for i, _ in a}) > 1  # the labeled fraction varies over targets


def test_planted_problem_has_the_planted_counts_and_a_valid_graph():
    """Feature f occurs in exactly counts[f] distinct samples (a count of n: every sample);
    columns strictly increase in a row; the path graph is symmetric with degrees 1 and 2 and
    no self loops; both classes are labeled."""
    counts = [50, 20, 7, 1, 0, 3]
    pb = synth.planted_problem(50, counts, n_lab=10, pos_frac=0.3, seed=3)
    assert pb.d == len(counts) and pb.n == 50
    assert np.array_equal(np.bincount(pb.x_col, minlength=pb.d), counts)
    for i in range(pb.n):
        row = pb.x_col[pb.x_rowptr[i]:pb.x_rowptr[i + 1]]
        assert np.all(np.diff(row) > 0) and row[0] == 0  # feature 0 is in every sample
    deg = np.diff(pb.s_rowptr)
    assert deg[0] == deg[-1] == 1 and np.all(deg[1:-1] == 2)
    src = np.repeat(np.arange(pb.n), deg)
    edges = set(zip(src.tolist(), pb.s_col.tolist()))
    assert all((j, i) in edges for i, j in edges) and all(i != j for i, j in edges)
    assert all(abs(i - j) == 1 for i, j in edges)
    assert pb.lab_idx.size == 10 and np.all(np.diff(pb.lab_idx) > 0)
    assert set(np.unique(pb.lab_y).tolist()) == {-1, 1} and int((pb.lab_y == 1).sum()) == 3
