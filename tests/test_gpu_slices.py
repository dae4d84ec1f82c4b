"""The sliced plans of the X^T product vs the CPU oracle and vs the unsliced plan.

LDS slices (n <= 262,144) and the hybrid of LDS slices for the longest rows and XCD
slices for the other split rows (larger n) are chosen automatically; FSDA_XT_SLICES=lds,
8, hyb or 1 forces LDS slices, XCD slices, the hybrid or no slices, which is how these
tests run the plans on the same inputs.  Split rows are summed in a different order than in
the unsliced plan, so the plans agree to rounding (1e-13 relative on products) but are not
bit-identical; the oracle bars are those of the unsliced parity tests.

The planted problems (24 features with fixed row lengths of X^T) cover every part of each
plan.  XCD slices, 300,000 samples: a dense feature whose slices are longer than one chunk
(two rounds of chunk items, the second ones short), the other chunk-summed rows (>= 8192
nonzeros), each bin of split rows ([1024, 8192), [512, 1024), [256, 512), [64, 256)).  LDS
slices, 200,000 samples (25 slices of 8192): rows in each bin by expected segment length
(>= 256, >= 64, >= 16 nonzeros per slice, and fewer), a dense feature.  Both: the short and
empty rows that stay unsplit.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
fsda = pytest.importorskip("paper_1709_04794_amd")

pytestmark = pytest.mark.gpu

PLANTED_COUNTS = [300000, 120000, 20000, 9000, 5000, 3000, 1500, 800, 600, 400, 300, 200, 100, 80, 64,
                  63, 40, 20, 10, 5, 2, 1, 0, 0]
# FSDA_XT_SLICES of each plan; the hybrid plan (rows of at least a head length in
# LDS slices, the other split rows in XCD slices) with its default head of 512
# nonzeros, a head of 64 (every split row in LDS slices, none left to XCD slices)
# and of 50,000 (the XCD part keeps rows of >= 8192 nonzeros, summed in chunk items)
PLANS = ["8", "lds", "hyb", "hyb64", "hyb50k"]
HEADS = {"hyb": None, "hyb64": "64", "hyb50k": "50000"}


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rhs_term_scale(pb, r):
    """Per feature, the sum of the magnitudes of the terms of the Alg. 7 right-hand side
    (X - 1 mu_l^T)^T v with v = [W 0; 0 0] X r (on a labeled sample, the mean of X r over
    its class; 0 elsewhere): entries whose terms cancel (a feature present in every
    sample has a zero centred column) are exact only to rounding of this size."""
    t = np.zeros(pb.n)
    rows = np.repeat(np.arange(pb.n), np.diff(pb.x_rowptr))
    np.add.at(t, rows, r[pb.x_col])
    v = np.zeros(pb.n)
    for c in (1, -1):
        m = pb.lab_y == c
        v[pb.lab_idx[m]] = t[pb.lab_idx[m]].mean()
    xtv = np.zeros(pb.d)
    np.add.at(xtv, pb.x_col, np.abs(v)[rows])
    lab = np.zeros(pb.n, bool)
    lab[pb.lab_idx] = True
    mu = np.bincount(pb.x_col[lab[rows]], minlength=pb.d) / pb.lab_idx.size
    return xtv + mu * np.abs(v).sum()


def build(pb, monkeypatch, slices, **kw):
    slices = str(slices)
    monkeypatch.setenv("FSDA_XT_SLICES", "hyb" if slices in HEADS else slices)
    if HEADS.get(slices):
        monkeypatch.setenv("FSDA_XT_HEAD", HEADS[slices])
    else:
        monkeypatch.delenv("FSDA_XT_HEAD", raising=False)
    return fsda.Operator.from_problem(pb, **kw)


@pytest.fixture(scope="module")
def tiny():
    return synth.workload("tiny")


@pytest.fixture(scope="module")
def planted_by_plan():
    """XCD slices: 300,000 samples; LDS slices: 200,000 (a dense feature of 200,000)."""
    xcd = synth.planted_problem(300000, PLANTED_COUNTS, n_lab=3000, pos_frac=0.3, alpha=0.5,
                                betas=(0.05, 0.5, 5.0, 50.0), seed=4, rtol=1e-11)
    return {"8": xcd, "hyb": xcd, "hyb64": xcd, "hyb50k": xcd,
            "lds": synth.planted_problem(200000, [200000] + PLANTED_COUNTS[1:], n_lab=2000, pos_frac=0.3,
                                         alpha=0.5, betas=(0.05, 0.5, 5.0, 50.0), seed=6, rtol=1e-11)}


@pytest.mark.parametrize("plan", PLANS)
@pytest.mark.parametrize("which", ["tiny", "planted"])
def test_sliced_products_match_oracle_and_unsliced(tiny, planted_by_plan, monkeypatch, which, plan):
    pb = tiny if which == "tiny" else planted_by_plan[plan]
    op8 = build(pb, monkeypatch, plan)
    op1 = build(pb, monkeypatch, 1)
    p = synth.normal(pb.d, seed=2, stream=3)
    for sigma in (0.0, 1e-2):
        q8 = op8.apply(sigma, torch.from_numpy(p).cuda())
        q1 = op1.apply(sigma, torch.from_numpy(p).cuda())
        ref = oracle.apply(pb, sigma, p)
        assert maxrel(q8.cpu().numpy(), ref) < 1e-12, sigma
        assert maxrel(q8.cpu().numpy(), q1.cpu().numpy()) < 1e-13, sigma
        if which == "planted":  # the two plans really differ (summation order of the split rows)
            assert not torch.equal(q8, q1)
    b8 = op8.rhs().cpu().numpy()
    assert maxrel(b8, oracle.rhs(pb)) < 1e-13
    r = synth.normal(pb.d, seed=3, stream=1)
    br = op8.rhs(torch.from_numpy(r).cuda()).cpu().numpy()
    ref = oracle.rhs(pb, r)
    tol = 1e-11 * np.abs(ref).max() + 1e-13 * rhs_term_scale(pb, r)
    assert (np.abs(br - ref) <= tol).all(), np.abs(br - ref) / tol


@pytest.mark.parametrize("plan", PLANS)
@pytest.mark.parametrize("alpha", [1.0, 0.5, 0.0])
def test_sliced_solve_matches_oracle_tiny(tiny, monkeypatch, alpha, plan):
    op = build(tiny, monkeypatch, plan, alpha=alpha)
    W, iters, relres, st = op.solve(tiny.betas, rtol=tiny.rtol)
    assert st == fsda.OK
    Wr, *_ = oracle.solve(tiny, rtol=1e-13, maxit=20000, alpha=alpha)
    W = W.cpu().numpy()
    b = oracle.rhs(tiny)
    for s, beta in enumerate(tiny.betas):
        assert relerr(W[s], Wr[s]) < 1e-6, (s, relerr(W[s], Wr[s]))
        assert relres[s] < 20 * tiny.rtol
        ref = np.linalg.norm(b - oracle.apply(tiny, beta, W[s], alpha=alpha)) / np.linalg.norm(b)
        assert abs(relres[s] - ref) <= 1e-3 * ref + 1e-15


@pytest.mark.parametrize("plan", PLANS)
@pytest.mark.parametrize("chunk", [1, 3, 128])
def test_sliced_solve_planted_matches_oracle(planted_by_plan, monkeypatch, chunk, plan):
    """Fold interval 1 puts r_i and r_{i+1} in one ring slot (the split rows are read and
    written by k_assemble); 3 and 128 end the solve inside a fold interval, after which no
    kernel of the remaining iterations may write the ring."""
    planted = planted_by_plan[plan]
    op = build(planted, monkeypatch, plan, max_chunk=128)
    W, iters, relres, st = op.solve(planted.betas, rtol=planted.rtol, chunk=chunk)
    assert st == fsda.OK
    Wr, itr, *_ = oracle.solve(planted, rtol=1e-13, maxit=20000)
    W = W.cpu().numpy()
    for s in range(planted.betas.size):
        assert relerr(W[s], Wr[s]) < 1e-6, (s, relerr(W[s], Wr[s]))
        assert relres[s] < 20 * planted.rtol
    W1, it1, *_ = build(planted, monkeypatch, plan, max_chunk=128).solve(planted.betas, rtol=planted.rtol, chunk=1)
    assert np.array_equal(iters, it1)
    assert maxrel(W, W1.cpu().numpy()) < 1e-12


@pytest.mark.parametrize("plan", PLANS)
def test_sliced_solve_is_deterministic_and_graph_equals_direct(planted_by_plan, monkeypatch, plan):
    """Replays of the captured fold interval give the same bits as direct launches."""
    planted = planted_by_plan[plan]
    op_g = build(planted, monkeypatch, plan)
    monkeypatch.setenv("FSDA_NO_GRAPH", "1")
    op_d = build(planted, monkeypatch, plan)
    monkeypatch.delenv("FSDA_NO_GRAPH")
    for _ in range(3):  # replays with eager work in between
        Wg, itg, rg, _ = op_g.solve(planted.betas, rtol=planted.rtol, chunk=16)
        Wd, itd, rd, _ = op_d.solve(planted.betas, rtol=planted.rtol, chunk=16)
        torch.cuda.synchronize()
        assert torch.equal(Wg, Wd)
        assert np.array_equal(itg, itd)
        assert np.array_equal(rg, rd)


@pytest.mark.parametrize("plan", PLANS)
def test_sliced_regression_and_mixed_tiny(tiny, monkeypatch, plan):
    z = synth.normal(tiny.n, seed=3, stream=8)
    betas = np.logspace(-2, 2, 6)
    op = build(tiny, monkeypatch, plan)
    W, iters, relres, st = op.regression_solve(torch.from_numpy(z).cuda(), betas, rtol=1e-10)
    assert st == fsda.OK
    Wr, *_ = oracle.reg_solve(tiny, z, betas, rtol=1e-13, maxit=50000)
    for s in range(betas.size):
        assert relerr(W[s].cpu().numpy(), Wr[s]) < 1e-6, s
    opm = build(tiny, monkeypatch, plan, precision=fsda.MIXED)
    Wm, itm, rm, stm = opm.solve(tiny.betas, rtol=1e-8)
    assert stm == fsda.OK
    Wo, *_ = oracle.solve(tiny, rtol=1e-13, maxit=20000)
    for s in range(tiny.betas.size):
        assert relerr(Wm[s].cpu().numpy(), Wo[s]) < 1e-4, s
        assert rm[s] <= 1e-8


@pytest.mark.parametrize("plan", PLANS)
@pytest.mark.parametrize("n", [3, 7, 9, 70, 130])
def test_sliced_tiny_sample_counts(monkeypatch, n, plan):
    """Fewer samples than slices (empty slices), n not a multiple of 8, a dense feature and
    features of 64 and more samples (split rows in every bin that fits), empty features."""
    counts = [n, max(1, n // 2), min(n, 64), min(n, 65), 2, 1, 0]
    pb = synth.planted_problem(n, counts, n_lab=max(2, n // 3), pos_frac=0.4, alpha=0.6,
                               betas=(1e-2, 0.3, 4.0), seed=n, rtol=1e-11)
    op = build(pb, monkeypatch, plan)
    p = synth.normal(pb.d, seed=n, stream=2)
    q = op.apply(1e-2, torch.from_numpy(p).cuda()).cpu().numpy()
    ref = oracle.apply(pb, 1e-2, p)
    assert maxrel(q, ref) < 1e-12
    W, iters, relres, st = op.solve(pb.betas, rtol=pb.rtol)
    assert st == fsda.OK
    Wr, *_ = oracle.solve(pb, rtol=1e-13, maxit=50000)
    for s in range(pb.betas.size):
        assert relerr(W[s].cpu().numpy(), Wr[s]) < 1e-6, (n, s)
