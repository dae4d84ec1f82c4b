"""Seeded synthetic inputs for the semi-supervised discriminant analysis (SDA) solve.

This module generates inputs only: a sparse binary fingerprint-like matrix X
(index-only CSR), a labeled subset with +-1 labels, a binary symmetric
Tanimoto k-nearest-neighbour similarity graph S (index-only CSR, no self
loops), a grid of regularisation shifts and, when asked, the uniform random
start vector that the paper's FSDA algorithm draws (Alg. 7, second step).
It holds none of the solver's arithmetic, so both the CPU oracle and the GPU
path consume exactly the same arrays.

Shapes follow the paper's workloads: sparse binary ECFP fingerprints
(Sec. 5.1, Table "characteristics of the ChEMBL data matrix": ~73 nonzeros per
row), a labeled fraction of a few percent (Table of the chosen ChEMBL
targets), a k-nearest-neighbour graph under Tanimoto similarity (Sec. 2.4 and
Sec. 5.1) and a log-spaced grid of regularisation values (Sec. 5.1).
The real ChEMBL / Janssen data are not available; these arrays stand in for
them.

The heavy loops live in ``synth.c`` (OpenMP, counter-based RNG so results do
not depend on the thread count).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import time
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``synth.c`` into ``libsynth.so`` next to it."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "synth.c")
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", src,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        U64 = ctypes.c_uint64
        lib.synth_fp_rowlen.argtypes = [I64, I64, ctypes.c_double, U64, P]
        lib.synth_permutation.argtypes = [I64, U64, U64, P]
        lib.synth_fp_fill.argtypes = [I64, I64, P, P, P, U64, P]
        lib.synth_knn_exact.argtypes = [I64, P, P, ctypes.c_int, ctypes.c_int, I64, P, P]
        lib.synth_knn_lsh.argtypes = [I64, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, U64, I64, P, P]
        lib.synth_normal.argtypes = [I64, U64, U64, P]
        lib.synth_uniform.argtypes = [I64, ctypes.c_double, ctypes.c_double, U64, U64, P]
        for f in (lib.synth_fp_rowlen, lib.synth_permutation, lib.synth_fp_fill, lib.synth_knn_exact,
                  lib.synth_knn_lsh, lib.synth_normal, lib.synth_uniform):
            f.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


# ---------------------------------------------------------------------------
# fingerprints
# ---------------------------------------------------------------------------

def fingerprints(n: int, d: int, mean_nnz: float, zipf_s: float, seed: int):
    """Binary matrix X (n x d) as (rowptr int32[n+1], col int32[nnz]).

    Row i has max(1, Poisson(mean_nnz)) distinct features; features are drawn
    with weight 1/rank**zipf_s without replacement, rank mapped through a
    seeded permutation of feature ids.  Columns sorted within each row.
    """
    lib = _load()
    rp64 = np.zeros(n + 1, dtype=np.int64)
    lib.synth_fp_rowlen(n, d, float(mean_nnz), seed, _ptr(rp64))
    nnz = int(rp64[-1])
    if nnz >= 2 ** 31:
        raise ValueError("nnz does not fit int32")
    w = 1.0 / np.power(np.arange(1, d + 1, dtype=np.float64), zipf_s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    cdf[-1] = 1.0
    perm = np.empty(d, dtype=np.int32)
    lib.synth_permutation(d, seed, 3, _ptr(perm))
    col = np.empty(nnz, dtype=np.int32)
    lib.synth_fp_fill(n, d, _ptr(rp64), _ptr(cdf), _ptr(perm), seed, _ptr(col))
    return rp64.astype(np.int32), col


# ---------------------------------------------------------------------------
# similarity graph
# ---------------------------------------------------------------------------

def _symmetrize(n: int, nbr: np.ndarray, cnt: np.ndarray):
    """Union of directed neighbour lists with their transpose -> CSR, no self loops."""
    cap = nbr.shape[1]
    mask = np.arange(cap)[None, :] < cnt[:, None]
    src = np.repeat(np.arange(n, dtype=np.int64), cnt.astype(np.int64))
    dst = nbr[mask].astype(np.int64)
    keys = np.concatenate([src * n + dst, dst * n + src])
    keys = np.unique(keys)
    r = keys // n
    c = keys % n
    keep = r != c
    r, c = r[keep], c[keep]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr.astype(np.int32), c.astype(np.int32)


EXACT_KNN_MAX = 20000  # "auto" builds the exact graph up to this many samples, MinHash LSH beyond


def knn_graph(n: int, x_rowptr: np.ndarray, x_col: np.ndarray, k: int, ties: bool = True,
              method: str = "auto", seed: int = 0, cap: Optional[int] = None):
    """Binary symmetric k-NN graph under Tanimoto similarity (Sec. 2.4).

    ``ties=True`` links a row to every row at least as similar as its k-th
    nearest neighbour (the paper links each point to all points within the
    k-th neighbour's distance).  ``method`` is "exact" (all pairs), "lsh"
    (MinHash candidates + exact re-rank, for large n) or "auto".
    Returns (rowptr int32[n+1], col int32[nnz]), sorted columns.
    """
    if k <= 0:  # no graph
        return np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32)
    lib = _load()
    rp = np.ascontiguousarray(x_rowptr, dtype=np.int64)
    col = np.ascontiguousarray(x_col, dtype=np.int32)
    if method == "auto":
        method = "exact" if n <= EXACT_KNN_MAX else "lsh"
    if cap is None:
        cap = max(4 * k, 64)
    nbr = np.zeros((n, cap), dtype=np.int32)
    cnt = np.zeros(n, dtype=np.int64)
    if method == "exact":
        lib.synth_knn_exact(n, _ptr(rp), _ptr(col), k, int(ties), cap, _ptr(nbr), _ptr(cnt))
    elif method == "lsh":
        lib.synth_knn_lsh(n, _ptr(rp), _ptr(col), k, int(ties), 12, 2, 6, seed, cap, _ptr(nbr), _ptr(cnt))
    else:
        raise ValueError(method)
    return _symmetrize(n, nbr, cnt)


def normal(n: int, seed: int, stream: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _load().synth_normal(n, seed, stream, _ptr(out))
    return out


def uniform(n: int, lo: float, hi: float, seed: int, stream: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _load().synth_uniform(n, lo, hi, seed, stream, _ptr(out))
    return out


# ---------------------------------------------------------------------------
# labels
# ---------------------------------------------------------------------------

def labels(n: int, x_rowptr: np.ndarray, x_col: np.ndarray, d: int, n_lab: int, pos_frac: float, seed: int):
    """Labeled rows and +-1 labels.

    ``n_lab`` rows are chosen uniformly without replacement; among them the
    top ``pos_frac`` fraction by a hidden linear score sum_{j in row} h_j,
    h ~ N(0,1)^d, are positive (a planted linear signal), the rest negative.
    Returns (lab_idx int32 sorted, lab_y int8).
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 77]))
    lab_idx = np.sort(rng.choice(n, size=n_lab, replace=False)).astype(np.int32)
    h = normal(d, seed, 11)
    # scores of the labeled rows only: each row's values gathered contiguously,
    # one reduction per row
    rp = x_rowptr.astype(np.int64)
    beg, lens = rp[lab_idx], rp[lab_idx + 1] - rp[lab_idx]
    off = np.zeros(n_lab + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    pos = np.repeat(beg - off[:-1], lens) + np.arange(off[-1])
    vals = h[x_col[pos]]
    s_lab = np.zeros(n_lab)
    nz = lens > 0
    if vals.size:
        s_lab[nz] = np.add.reduceat(vals, off[:-1][nz])
    n_pos = int(round(pos_frac * n_lab))
    n_pos = min(max(n_pos, 1), n_lab - 1)
    order = np.argsort(-s_lab, kind="stable")
    y = -np.ones(n_lab, dtype=np.int8)
    y[order[:n_pos]] = 1
    return lab_idx, y


def target_labels(pb, ntarget: int, seed: int, frac_median: float = 0.007, frac_sigma: float = 0.8,
                  frac_lo: float = 0.001, frac_hi: float = 0.05, pos_lo: float = 0.02, pos_hi: float = 0.30,
                  min_lab: int = 4):
    """Labeled sets of ``ntarget`` binary targets over the samples of ``pb``.

    Target c labels a fraction f_c of the samples, ln f_c ~ N(ln frac_median,
    frac_sigma) clipped to [frac_lo, frac_hi] (at least ``min_lab`` rows), with
    a positive rate ~ U(pos_lo, pos_hi); rows and signs come from ``labels``
    with a target-specific hidden score.  Returns a list of (lab_idx, lab_y).
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 91]))
    out = []
    for c in range(ntarget):
        f = float(np.clip(np.exp(rng.normal(np.log(frac_median), frac_sigma)), frac_lo, frac_hi))
        pos = float(rng.uniform(pos_lo, pos_hi))
        n_lab = min(pb.n, max(min_lab, int(round(f * pb.n))))
        out.append(labels(pb.n, pb.x_rowptr, pb.x_col, pb.d, n_lab, pos, seed=seed * 1000 + c + 1))
    return out


def holdout_splits(targets, seed: int, frac_ho: float = 0.2):
    """Splits each target's labeled set (``target_labels`` output) into a
    training part and a held-out part of round(frac_ho l) rows (at least one),
    keeping both classes in the training part.  Returns (train, heldout): lists
    of (lab_idx int32, lab_y int8) and (ho_idx int32 sorted, ho_y float64 +-1)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 77]))
    train, held = [], []
    for li, ly in targets:
        li, ly = np.asarray(li), np.asarray(ly)
        l = li.size
        nho = min(max(1, int(round(frac_ho * l))), l - 2)
        for _ in range(100):
            perm = rng.permutation(l)
            tr, ho = np.sort(perm[nho:]), np.sort(perm[:nho])
            if (ly[tr] > 0).any() and (ly[tr] < 0).any():
                break
        else:  # pragma: no cover - a labeled set with one example of a class
            raise ValueError("cannot keep both classes in the training part")
        train.append((li[tr].astype(np.int32), ly[tr].astype(np.int8)))
        o = np.argsort(li[ho], kind="stable")
        held.append((li[ho][o].astype(np.int32), ly[ho][o].astype(np.float64)))
    return train, held


# ---------------------------------------------------------------------------
# problems
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    """One SDA problem: X, graph S, labeled rows, alpha, shift grid."""
    name: str
    n: int
    d: int
    x_rowptr: np.ndarray
    x_col: np.ndarray
    s_rowptr: np.ndarray
    s_col: np.ndarray
    lab_idx: np.ndarray
    lab_y: np.ndarray
    alpha: float
    betas: np.ndarray
    rtol: float
    seed: int = 0

    @property
    def x_nnz(self) -> int:
        return int(self.x_col.size)

    @property
    def s_nnz(self) -> int:
        return int(self.s_col.size)

    def summary(self) -> dict:
        return {"n": self.n, "d": self.d, "nnz_x": self.x_nnz, "nnz_s": self.s_nnz,
                "n_lab": int(self.lab_idx.size), "n_pos": int((self.lab_y > 0).sum()),
                "alpha": self.alpha, "n_shift": int(self.betas.size), "rtol": self.rtol}


@dataclasses.dataclass
class Recipe:
    n: int
    d: int
    mean_nnz: float
    zipf_s: float
    lab_frac: float
    pos_frac: float
    k: int
    alpha: float
    betas: tuple
    rtol: float
    ties: bool = True
    knn: str = "auto"


# The workloads: tiny (parity), mid (the benchmark), large (fingerprint-shaped).
RECIPES = {
    "tiny": Recipe(n=2000, d=4096, mean_nnz=40, zipf_s=1.1, lab_frac=0.1, pos_frac=0.2, k=8, alpha=1.0,
                   betas=tuple(np.logspace(-2, 2, 8)), rtol=1e-10),
    "mid": Recipe(n=200_000, d=1_000_000, mean_nnz=60, zipf_s=1.1, lab_frac=0.02, pos_frac=0.1, k=10,
                  alpha=1.0, betas=tuple(np.logspace(-3, 2, 16)), rtol=1e-8),
    "large": Recipe(n=1_500_000, d=4_000_000, mean_nnz=70, zipf_s=1.2, lab_frac=0.01, pos_frac=0.05, k=10,
                    alpha=1.0, betas=tuple(np.logspace(-4, 2, 32)), rtol=1e-8),
    # the differentiation workload: 64 targets (labeled sets drawn by
    # target_labels, each split 80/20 by holdout_splits) over this X and graph;
    # alpha inside (0, 1) so that the alpha-derivative has both sides
    "diff": Recipe(n=500_000, d=2_000_000, mean_nnz=60, zipf_s=1.1, lab_frac=0.007, pos_frac=0.1, k=10,
                   alpha=0.9, betas=tuple(np.logspace(-3, 2, 8)), rtol=1e-8),
    # the shape of the ChEMBL matrix of the shifted-CG timing table (regression
    # phase only, so no graph): 167,668 x 291,714 with about 12.2 million nonzeros
    "chembl": Recipe(n=167_668, d=291_714, mean_nnz=72.8, zipf_s=1.1, lab_frac=0.01, pos_frac=0.2, k=0,
                     alpha=1.0, betas=tuple(10.0 ** np.arange(-9, 3)), rtol=1e-3),
}


def make_problem(recipe: Recipe, seed: int = 0, name: str = "custom", log=None, **override) -> Problem:
    """Generate a problem from a recipe; ``log`` (a callable taking one string), when given,
    is told when each of the three generation steps has finished."""
    r = dataclasses.replace(recipe, **override) if override else recipe
    t0 = time.perf_counter()

    def step(what):
        if log is not None:
            log("%s: %s done after %.1f s" % (name, what, time.perf_counter() - t0))

    xr, xc = fingerprints(r.n, r.d, r.mean_nnz, r.zipf_s, seed)
    step("fingerprints")
    sr, sc = knn_graph(r.n, xr, xc, r.k, ties=r.ties, method=r.knn, seed=seed)
    step("kNN graph")
    n_lab = max(2, int(round(r.lab_frac * r.n)))
    li, ly = labels(r.n, xr, xc, r.d, n_lab, r.pos_frac, seed)
    step("labels")
    return Problem(name=name, n=r.n, d=r.d, x_rowptr=xr, x_col=xc, s_rowptr=sr, s_col=sc, lab_idx=li,
                   lab_y=ly, alpha=float(r.alpha), betas=np.asarray(r.betas, dtype=np.float64), rtol=r.rtol,
                   seed=seed)


def workload(name: str, seed: int = 0, cache_dir: Optional[str] = None, log=None, **override) -> Problem:
    """Named workload; cached as .npz under ``cache_dir`` when given."""
    recipe = RECIPES[name]
    path = None
    if cache_dir is not None and not override:
        os.makedirs(cache_dir, exist_ok=True)
        path = os.path.join(cache_dir, "%s_s%d.npz" % (name, seed))
        if os.path.exists(path):
            z = np.load(path)
            return Problem(name=name, n=int(z["n"]), d=int(z["d"]), x_rowptr=z["x_rowptr"], x_col=z["x_col"],
                           s_rowptr=z["s_rowptr"], s_col=z["s_col"], lab_idx=z["lab_idx"], lab_y=z["lab_y"],
                           alpha=float(z["alpha"]), betas=z["betas"], rtol=float(z["rtol"]), seed=seed)
    pb = make_problem(recipe, seed=seed, name=name, log=log, **override)
    if path is not None:
        np.savez(path, n=pb.n, d=pb.d, x_rowptr=pb.x_rowptr, x_col=pb.x_col, s_rowptr=pb.s_rowptr,
                 s_col=pb.s_col, lab_idx=pb.lab_idx, lab_y=pb.lab_y, alpha=pb.alpha, betas=pb.betas,
                 rtol=pb.rtol)
    return pb


def planted_problem(n: int, counts, n_lab: int, pos_frac: float = 0.3, alpha: float = 0.5,
                    betas=(0.1, 1.0, 10.0), seed: int = 0, rtol: float = 1e-10) -> Problem:
    """X with planted feature counts: feature f occurs in counts[f] distinct samples drawn
    uniformly (counts[f] == n makes a dense column), so the rows of X^T have exactly these
    lengths.  The graph is the path i -- i+1 (symmetric, degrees 1 and 2).  n_lab labeled
    samples drawn uniformly, round(pos_frac n_lab) of them positive (at least one of each)."""
    rng = np.random.default_rng(seed)
    rs, cs = [], []
    for f, c in enumerate(counts):
        if c > 0:
            rs.append(np.arange(n) if c >= n else rng.choice(n, size=int(c), replace=False))
            cs.append(np.full(min(int(c), n), f))
    r = np.concatenate(rs) if rs else np.zeros(0, np.int64)
    c = np.concatenate(cs) if cs else np.zeros(0, np.int64)
    o = np.lexsort((c, r))
    x_rowptr = np.zeros(n + 1, np.int32)
    np.cumsum(np.bincount(r, minlength=n), out=x_rowptr[1:])
    x_col = c[o].astype(np.int32)
    left = np.arange(1, n)  # sample i > 0 links to i - 1, sample i < n - 1 to i + 1
    deg = np.full(n, 2, np.int64)
    deg[0] = deg[-1] = 1
    s_rowptr = np.zeros(n + 1, np.int32)
    np.cumsum(deg, out=s_rowptr[1:])
    s_col = np.empty(int(deg.sum()), np.int32)
    s_col[s_rowptr[left]] = left - 1
    right = np.arange(0, n - 1)
    s_col[s_rowptr[right + 1] - 1] = right + 1
    lab_idx = np.sort(rng.choice(n, size=n_lab, replace=False)).astype(np.int32)
    npos = min(max(1, int(round(pos_frac * n_lab))), n_lab - 1)
    lab_y = -np.ones(n_lab, np.int8)
    lab_y[rng.choice(n_lab, size=npos, replace=False)] = 1
    return Problem(name="planted", n=n, d=len(counts), x_rowptr=x_rowptr, x_col=x_col, s_rowptr=s_rowptr,
                   s_col=s_col, lab_idx=lab_idx, lab_y=lab_y, alpha=float(alpha),
                   betas=np.asarray(betas, dtype=np.float64), rtol=rtol, seed=seed)


def small_problem(n: int, d: int, mean_nnz: float = 6, k: int = 3, n_lab: Optional[int] = None,
                  pos_frac: float = 0.3, alpha: float = 0.5, betas=(1e-2, 1e-1, 1.0, 10.0), seed: int = 0,
                  zipf_s: float = 1.1, ties: bool = True, rtol: float = 1e-12) -> Problem:
    """A small random problem for tests (exact kNN)."""
    if n_lab is None:
        n_lab = max(2, n // 4)
    rec = Recipe(n=n, d=d, mean_nnz=mean_nnz, zipf_s=zipf_s, lab_frac=n_lab / n, pos_frac=pos_frac, k=k,
                 alpha=alpha, betas=tuple(betas), rtol=rtol, ties=ties, knn="exact")
    return make_problem(rec, seed=seed, name="small")
