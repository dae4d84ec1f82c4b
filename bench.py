"""Benchmark: shifted SDA solves per second on one MI355X.

Default run (the many-targets workload): a step is one call of
fsda_multishift_solve_batch on 64 binary targets over the mid-scale X and kNN
graph (200,000 x 1,000,000, 16 shifts each): per target its right-hand side,
its shifted CG over all 16 shifts (FP64) and the FP64 true residual of every
(target, shift).  Successive steps take the next 64 of 1000 targets (labeled
fraction lognormal around 0.7 %, positive rate U(0.02, 0.3)).  The value is
(target, shift) solves whose true relative residual is <= 1e-8, per second.
Beside it: the plain per-target FP64 path on the same X (one labeled set, one
multi-shift solve), and the roofline of the operator apply measured on the
large workload (1.5e6 x 4e6, 1.05e8 nonzeros; its vectors outgrow the
Infinity Cache), every launch of each apply kernel bracketed by HIP events.
Prints one JSON line.

    python bench.py [--steps K] [--warmup W]
    python bench.py --workload mid|large|tiny   # the single-target path of one workload

A separate mode replays the paper's CG versus shifted CG table on a matrix of
the ChEMBL shape:

    python bench.py --experiment shifted-table
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TARGET_RELRES = 1e-8
# The solvers stop on their recursive residual; they are asked for 1 % below the
# counted threshold, so that rounding drift between it and the true FP64 residual
# (a relative 1e-6 of the threshold has been seen) does not fail a solve.  This
# costs about one iteration per solve.
SOLVE_RTOL = 0.99 * TARGET_RELRES


def log(*a):
    print(*a, file=sys.stderr, flush=True)


LSLICE, MAXLSLICE, SPLIT_ROW, XCD_SPLIT_ROW, LDS_HEAD = 8192, 32, 64, 16, 512  # the X^T plans of the library


def xt_plan(pb):
    """The X^T plan the library picks for this problem (and FSDA_XT_SLICES, FSDA_XT_HEAD):
    a dict with the plan ("lds", "xcd", "hyb" or "none"), the LDS slice count, and the
    rows of X^T in LDS slices and in XCD slices (counts and nonzeros)."""
    cnt = np.bincount(pb.x_col, minlength=pb.d)
    nl = -(-pb.n // LSLICE)
    env = os.environ.get("FSDA_XT_SLICES", "")
    head = max(int(os.environ.get("FSDA_XT_HEAD", LDS_HEAD)), SPLIT_ROW)
    if env == "1":
        plan = "none"
    elif env == "8":
        plan = "xcd"
    elif env == "hyb":
        plan = "hyb"
    elif nl <= MAXLSLICE:
        plan = "lds"
    else:
        plan = "hyb" if 8 * pb.n > (2 << 20) else "none"
    split = cnt >= SPLIT_ROW
    lds = (cnt >= head) if plan == "hyb" else (split if plan == "lds" else np.zeros_like(split))
    xcd = (cnt >= XCD_SPLIT_ROW) & ~lds if plan in ("hyb", "xcd") else np.zeros_like(split)
    lens = cnt[xcd]
    xparts = int((8 * np.maximum(1, -(-(lens // 8) // 32768))).sum()) if lens.size else 0
    return {"plan": plan, "nsl": nl if plan in ("lds", "hyb") else 0,
            "n_lds": int(lds.sum()), "z_lds": int(cnt[lds].sum()), "n_xcd": int(xcd.sum()),
            "z_xcd": int(cnt[xcd].sum()), "xcd_parts": xparts}


def algorithmic_bytes(kernel: int, pb, nshift: int, chunk: int) -> float:
    """Bytes one launch must move (every array once; gathered vectors counted once; int32 indices)."""
    import paper_1709_04794_amd as fsda
    n, d, z, g = pb.n, pb.d, pb.x_nnz, pb.s_nnz
    lab = 8 * n if pb.alpha < 1.0 else 0
    pl = xt_plan(pb) if kernel in (fsda.K_XT, fsda.K_XTL, fsda.K_ASM) else None
    if kernel == fsda.K_XTL:    # LDS rows' indices and slice bounds, u (staged once per slice), parts written
        nsl, nr = pl["nsl"], pl["n_lds"]
        return float(4 * pl["z_lds"] + 4 * (nsl + 1) * nr + 8 * n + 8 * nsl * nr) if nr else 0.0
    if kernel == fsda.K_XT:     # the other rows' indices, u; p and r in, r out but for the XCD-split rows;
        # LDS parts read, XCD parts written
        return float(4 * (d + 1) + 4 * (z - pl["z_lds"]) + 8 * n + 24 * (d - pl["n_xcd"])
                     + 8 * pl["nsl"] * pl["n_lds"] + 8 * pl["xcd_parts"])
    if kernel == fsda.K_ASM:    # XCD slices: the split rows' parts in, then p and r in, r out per row
        nx = pl["n_xcd"]
        return float(8 * pl["xcd_parts"] + 4 * (nx + 1) + 24 * nx) if nx else 0.0
    if kernel == fsda.K_X:      # rowptr, col, p (gathered), t written
        return 4 * (n + 1) + 4 * z + 8 * d + 8 * n + lab
    if kernel == fsda.K_S:      # rowptr, col, t (gathered), u written
        return 4 * (n + 1) + 4 * g + 8 * n + 8 * n + lab
    if kernel == fsda.K_RESID:  # not launched by the feature-space solve
        return 0.0
    if kernel == fsda.K_PUPD:   # r_{i+1}, p in; p out (the long rows' chunk sums aside)
        return 24 * d
    if kernel == fsda.K_FOLD:   # W, P in and out for every shift, chunk residuals in
        return 32 * nshift * d + 8 * chunk * d
    return 0.0


TRAFFIC_KEYS = {2: "k_xt", 3: "k_xt_lds", 0: "k_rows_x", 6: "k_fold", 1: "k_rows_s", 13: "k_assemble"}


def kernel_source_key() -> str:
    """sha256 prefix of the device code (kernels.h without comments or blank lines): the
    byte counters in profiles/ hold for the kernels they were taken on."""
    import hashlib
    import re
    src = open(os.path.join(ROOT, "paper_1709_04794_amd", "csrc", "kernels.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in src.splitlines()]
    return hashlib.sha256("\n".join(ln for ln in lines if ln.strip()).encode()).hexdigest()[:16]


def measured_traffic(kernel: int, workload: str):
    """HBM bytes per launch from the committed rocprofv3 byte counters, if they
    were taken on the current kernel source; otherwise None."""
    import glob
    key = TRAFFIC_KEYS.get(kernel)
    if key is None:
        return None
    sha = kernel_source_key()
    for f in glob.glob(os.path.join(ROOT, "profiles", "*traffic*.txt")):
        for line in open(f):
            if not line.startswith("TRAFFIC "):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            if kv.get("kernel") == key and kv.get("workload") == workload and kv.get("source") == sha:
                return int(float(kv["bytes"]))
    return None


KNAMES = {0: "k_rows<EpiX> (t = X p)", 1: "k_rows<EpiLap> (u = M' t)",
          2: "k_xt<EpiXTR> (q = X^T u + s p, r -= a q)", 3: "k_xt_lds (X^T split rows from LDS slices)",
          4: "k_resid (sample space)",
          5: "k_pupdate (long rows of X^T, p update, shift scalars)", 6: "k_fold",
          13: "k_assemble<EpiXTR> (X^T split rows from their XCD-slice parts, r -= a q)"}
APPLY_CLASSES = (0, 1, 2, 3, 13)  # the kernels of one operator apply (X, graph, X^T and its parts)


def graph_stats(pb) -> dict:
    """How the workload's kNN graph was made and its degrees (the graph is an input of the solve)."""
    import synth
    deg = np.diff(pb.s_rowptr)
    exact = pb.n <= synth.EXACT_KNN_MAX
    return {"method": "exact Tanimoto kNN, ties included" if exact else
            "MinHash-LSH candidates re-ranked by exact Tanimoto, ties included (an approximation of the exact graph)",
            "neighbours_kept_per_sample_before_symmetrising": "at most max(4k, 64)",
            "mean_degree": round(float(deg.mean()), 2), "max_degree": int(deg.max()), "nnz": int(pb.s_nnz)}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def cpu_baseline(pb, budget_s: float):
    """The oracle (per-shift FP64 CG) on the host cores, on a bounded sample of shifts."""
    import oracle
    nt = oracle.max_threads()
    order = [int(np.argmax(pb.betas)), int(np.argmin(pb.betas))]
    solved, spent, sample = 0, 0.0, []
    for s in order:
        if spent > budget_s:
            break
        t0 = time.perf_counter()
        W, it, rel, rc = oracle.solve(pb, betas=[pb.betas[s]], rtol=pb.rtol, maxit=20000)
        dt = time.perf_counter() - t0
        spent += dt
        ok = bool(rel[0] <= TARGET_RELRES)
        solved += ok
        sample.append({"beta": float(pb.betas[s]), "iters": int(it[0]), "seconds": round(dt, 3),
                       "relres": float(rel[0])})
    return {"value": solved / spent if spent > 0 else 0.0, "unit": "solves/s", "cores": nt, "kind": "oracle",
            "sample": "per-shift FP64 CG of the oracle on the same %s workload for %d of its %d shifts "
                      "(largest and smallest beta) to rel. residual %.0e: %s"
                      % (pb.name, len(sample), pb.betas.size, pb.rtol, json.dumps(sample))}


def time_paths(pb, fsda, torch, chunk: int):
    """One warm and one timed call of each further entry point on the workload."""
    import synth
    out = {}
    S = pb.betas.size

    def timed(fn, reps=1):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, r

    op_m = fsda.Operator.from_problem(pb, precision=fsda.MIXED, max_chunk=chunk)
    dt, (W, it, rel, st) = timed(lambda: op_m.solve(pb.betas, rtol=SOLVE_RTOL, chunk=chunk))
    out["mixed"] = {"seconds": round(dt, 4), "solves_per_s": round(int((rel <= TARGET_RELRES).sum()) / dt, 3),
                    "worst_relres": float(rel.max()), "iters": it.tolist(), "status": st,
                    "what": "FP32 shared recurrence to 1e-5, then FP64 residuals and batched FP32 correction "
                            "solves, every shift to rel. residual %.0e" % pb.rtol}
    op_m.close()
    del op_m
    op = fsda.Operator.from_problem(pb, max_chunk=chunk)
    labs = synth.target_labels(pb, 16, seed=1)
    dt, (W, it, rel, st) = timed(lambda: op.solve_batch(labs, pb.betas, rtol=SOLVE_RTOL))  # its default fold interval
    out["batched_targets"] = {"targets": len(labs), "seconds": round(dt, 4),
                              "shifted_solves_per_s": round(int((rel <= TARGET_RELRES).sum()) / dt, 3),
                              "worst_relres": float(rel.max()), "max_iters": int(it.max()), "status": st,
                              "what": "16 labelings (labeled fraction lognormal around 0.7%%, positive rate "
                                      "U(0.02, 0.3)) x %d shifts, FP64, to rel. residual %.0e" % (S, pb.rtol)}
    del W
    dt, (Z, it, rel, st) = timed(lambda: op.sa_solve(pb.betas, rtol=SOLVE_RTOL, chunk=chunk), reps=3)
    out["sample_space"] = {"seconds": round(dt, 5), "solves_per_s": round(int((rel <= TARGET_RELRES).sum()) / dt, 3),
                           "worst_relres": float(rel.max()), "max_iters": int(it.max()), "status": st,
                           "what": "Alg. sasda ratings for every shift, FP64, to rel. residual %.0e" % pb.rtol}
    op.close()
    del op
    # hold-out loss of every shift and its gradient in (log beta, alpha) by the
    # adjoint method: forward solve, hold-out loss, batched adjoint solves, gradient
    from paper_1709_04794_amd import hyper
    rng = np.random.default_rng(3)
    pool = np.setdiff1d(np.arange(pb.n), pb.lab_idx)
    ho = np.sort(rng.choice(pool, size=min(2000, pool.size), replace=False))
    ho_y = np.where(synth.normal(ho.size, seed=3, stream=7) > 0, 1.0, -1.0)
    obj = hyper.Objective(pb, ho, ho_y, rtol=pb.rtol)
    lb = torch.tensor(np.log(pb.betas), dtype=torch.float64, requires_grad=True)
    al = torch.tensor(float(pb.alpha), dtype=torch.float64, requires_grad=True)

    def hypergrad():
        lb.grad = al.grad = None
        loss = hyper.HoldoutLoss.apply(lb, al, obj)
        loss.sum().backward()
        return loss

    dt, loss = timed(hypergrad)
    out["hypergradient"] = {"seconds": round(dt, 4), "shifts": S, "holdout_rows": int(ho.size),
                            "finite": bool(torch.isfinite(lb.grad).all() and torch.isfinite(al.grad)),
                            "what": "hold-out loss of %d shifts and its gradient in (log beta, alpha): forward solve, "
                                    "hold-out loss, %d adjoint solves (batched), gradient; FP64, rtol %.0e"
                                    % (S, S, pb.rtol)}
    for o in obj._ops.values():
        o.close()
    return out


SHIFTED_TABLE = [  # (betas, CG seconds, shifted CG seconds, speed-up) as printed in Table tab:shifted
    (tuple(10.0 ** np.arange(-9, 3)), 43.11, 6.02, 7.16),
    (tuple(np.round(np.arange(1.0, 2.15, 0.1), 1) * 1e-6), 50.98, 5.68, 8.98),
]


HOT_FEATURES = 8192  # features the X product reads from shared memory


def gather_patterns(pb):
    """Index streams of the three products (features in decreasing frequency, as
    the operator orders them): X^T gathers u at the samples of every feature
    row; X gathers p at the features of every sample beyond the ones staged in
    shared memory; S gathers t at the neighbours of every sample."""
    n, d = pb.n, pb.d
    cnt = np.bincount(pb.x_col, minlength=d)
    new = np.empty(d, np.int64)
    new[np.argsort(-cnt, kind="stable")] = np.arange(d)
    xrow = np.repeat(np.arange(n), np.diff(pb.x_rowptr))
    xcol = new[pb.x_col]
    o = np.lexsort((xrow, xcol))
    cold = xcol >= HOT_FEATURES
    short = cnt[pb.x_col[o]] < SPLIT_ROW  # rows of X^T left to L2 gathers by the LDS-slice plan
    return {"xt": (xcol[o], xrow[o], n), "x_cold": (xrow[cold], xcol[cold], d),
            "xt_short": (xcol[o][short], xrow[o][short], n),
            "s": (np.repeat(np.arange(n), np.diff(pb.s_rowptr)), pb.s_col, n)}


def xcd_sliced_stream(idx, n, aligned=True, piece=256, nslice=8):
    """The X^T index stream (sample indices < n) reordered for fsda_gather_sum's
    grid-stride loop, where entry k is handled by block (k // piece) % grid and
    blocks go to the XCDs round robin: piece p holds only indices of sample slice
    p % nslice ([x n / nslice, (x+1) n / nslice)), so each XCD gathers from one
    slice.  aligned=False rotates the slice of each round of nslice pieces, so that
    every slice is spread over all XCDs (same pieces, same order within a slice).
    The leftover of the unequal slices follows at the end, unsliced."""
    idx = np.asarray(idx)
    sl = (idx.astype(np.int64) * nslice) // n
    o = np.argsort(sl, kind="stable")
    parts = np.split(idx[o], np.searchsorted(sl[o], np.arange(1, nslice)))
    m = min(len(q) for q in parts) // piece * piece
    A = np.stack([q[:m].reshape(-1, piece) for q in parts], axis=1)  # [round, slice, piece]
    if not aligned:
        R = A.shape[0]
        A = A[np.arange(R)[:, None], (np.arange(nslice)[None, :] + np.arange(R)[:, None]) % nslice]
    return np.concatenate([A.reshape(-1)] + [q[m:] for q in parts])


def time_gathers(fsda, torch, size, idx, reps=10, pair_us=0.0):
    """Best time (us) of the bare gather kernel over idx into a vector of `size`."""
    src = torch.rand(size, dtype=torch.float64, device="cuda")
    it = torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).cuda()
    part = fsda.gather_sum(src, it)  # checks the indices once
    want = float(src[it.long()].sum())
    got = float(part.sum())
    assert abs(got - want) <= 1e-9 * max(1.0, abs(want)), (got, want)
    best = 1e9
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fsda.gather_sum(src, it, part=part, checked=True)  # the kernel alone between the events
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) * 1e3 - pair_us)
    return best


def event_pair_us(torch, count=200):
    ev = []
    for _ in range(count):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        b.record()
        ev.append((a, b))
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev])) * 1e3


def gather_ceiling(args, fsda, torch):
    """The resource the sparse products are bound by: random 8-byte gathers.

    Times fsda_gather_sum (a bare gather-and-add kernel) on index streams of the
    workload's sizes: uniform indices, and the index patterns of the products
    themselves (X^T: the samples of every feature row; X: the features of every
    sample beyond the ones staged in shared memory; S: the neighbours of every
    sample), the X^T rows that the LDS-slice plan leaves to L2 gathers (rows of
    fewer than 64 nonzeros), and the X^T pattern cut into XCD slices
    (xcd_sliced_stream) with and without the alignment of slices to XCDs.  Also counts the distinct 128-byte lines each row of a product
    touches (16 FP64 values per line), the number of cache-line lookups a
    product cannot avoid.  Features are ordered by decreasing frequency, as the
    operator orders them internally.
    """
    import synth
    pb = synth.workload(args.workload, seed=args.seed, cache_dir=args.cache)
    n, d = pb.n, pb.d
    pat = gather_patterns(pb)

    def lines(rows, cols):
        return int(np.unique(rows.astype(np.int64) * (1 << 32) + cols // 16).size)

    stats = {"xt_entries": int(pat["xt"][1].size), "xt_lines": lines(*pat["xt"][:2]),
             "x_cold_entries": int(pat["x_cold"][1].size), "x_cold_lines": lines(*pat["x_cold"][:2]),
             "s_entries": int(pat["s"][1].size), "s_lines": lines(*pat["s"][:2])}
    log("distinct lines per row, summed: %s" % stats)
    rng = np.random.default_rng(args.seed)
    z = pat["xt"][1].size
    streams = {
        "uniform over n (u, t)": (n, rng.integers(0, n, z)),
        "X^T pattern over n (u)": (n, pat["xt"][1]),
        "uniform over d (p)": (d, rng.integers(0, d, z)),
        "X cold pattern over d (p)": (d, pat["x_cold"][1]),
        "S pattern over n (t)": (n, pat["s"][1]),
        "uniform over 4096 (L1-resident)": (4096, rng.integers(0, 4096, z)),
        "X^T short rows (LDS plan: L2 part)": (n, pat["xt_short"][1]),
        "X^T pattern, XCD slices": (n, xcd_sliced_stream(pat["xt"][1], n)),
        "X^T pattern, slices not XCD-aligned": (n, xcd_sliced_stream(pat["xt"][1], n, aligned=False)),
    }
    pair_us = event_pair_us(torch, 50)
    out = {}
    for name, (size, idx) in streams.items():
        best = time_gathers(fsda, torch, size, idx, pair_us=pair_us)
        out[name] = {"gathers": int(idx.size), "us": round(best, 2), "Ggathers_per_s": round(idx.size / best / 1e3, 1)}
        log("%-34s %9d gathers  %8.2f us  %6.1f G/s" % (name, idx.size, best, idx.size / best / 1e3))
    print(json.dumps({"experiment": "gather-ceiling", "workload": pb.name, "event_pair_us": round(pair_us, 2),
                      "lines": stats, "rates": out}))


# kernel classes of fsda_multishift_solve_batch (fsda_time_kernel)
BATCH_KNAMES = {7: "bX", 8: "bLap", 9: "bXT", 10: "bresid", 11: "bpupdate", 12: "tfold"}


def batched_targets(args, fsda, torch):
    """Many targets over one X and S (fsda_multishift_solve_batch): shifted solves per
    second at rel. residual 1e-8 for batches of 16, 32 and 64 labelings of the
    workload (labeled fraction lognormal around 0.7 %, positive rate U(0.02, 0.3)),
    with the tile chosen by fsda_batch_autotune."""
    import synth
    pb = synth.workload(args.workload, seed=args.seed, cache_dir=args.cache)
    op = fsda.Operator.from_problem(pb)
    # the tile (targets per pass over the indices) picked by the autotuner on the
    # first 16 labelings, then used for every batch below
    t0 = time.perf_counter()
    tile, groups, rates = op.autotune_batch(synth.target_labels(pb, 16, seed=1), pb.betas, trial_iters=32)
    tune = {"tile": tile, "groups_per_row": groups, "seconds": round(time.perf_counter() - t0, 2),
            "shifted_target_iterations_per_s": {"%dx%d" % sh: round(r, 1) for sh, r in rates.items()}}
    log("autotuned tile %d, %d groups per row, in %.1f s: %s" % (tile, groups, tune["seconds"],
                                                                tune["shifted_target_iterations_per_s"]))
    rows = []
    for k in (16, 32, 64):
        labs = synth.target_labels(pb, k, seed=1)
        op.solve_batch(labs[:4], pb.betas, rtol=SOLVE_RTOL, chunk=args.batch_chunk)  # warm the kernels
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        W, it, rel, st = op.solve_batch(labs, pb.betas, rtol=SOLVE_RTOL, chunk=args.batch_chunk)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        solved = int((rel <= TARGET_RELRES).sum())
        rows.append({"targets": k, "shifts": int(pb.betas.size), "seconds": round(dt, 3),
                     "shifted_solves_per_s": round(solved / dt, 2), "solved": solved,
                     "max_iters": int(it.max()), "worst_relres": float(rel.max()), "status": st})
        log("%d targets x %d shifts: %.3f s, %.1f shifted solves/s, worst relres %.2e"
            % (k, pb.betas.size, dt, solved / dt, rel.max()))
        del W
    many = None
    if args.targets > 0:  # e.g. 1000 targets in calls of 256 (the W of a call: 256 x 16 x d doubles)
        labs = synth.target_labels(pb, args.targets, seed=2)
        CALL = 256
        t0 = time.perf_counter()
        solved, worst, maxit = 0, 0.0, 0
        for c0 in range(0, args.targets, CALL):
            W, it, rel, st = op.solve_batch(labs[c0:c0 + CALL], pb.betas, rtol=SOLVE_RTOL, chunk=args.batch_chunk)
            torch.cuda.synchronize()
            solved += int((rel <= TARGET_RELRES).sum())
            worst, maxit = max(worst, float(rel.max())), max(maxit, int(it.max()))
            del W
            log("targets %d..%d done after %.1f s" % (c0, min(c0 + CALL, args.targets) - 1, time.perf_counter() - t0))
        dt = time.perf_counter() - t0
        many = {"targets": args.targets, "shifts": int(pb.betas.size), "seconds": round(dt, 2),
                "shifted_solves_per_s": round(solved / dt, 2), "solved": solved, "worst_relres": worst,
                "max_iters": maxit, "calls": -(-args.targets // CALL), "targets_per_call": CALL}
        log("%d targets x %d shifts: %.1f s, %.1f shifted solves/s" % (args.targets, pb.betas.size, dt, solved / dt))
    # per-kernel time of one 16-target solve: one solve per class, that class's
    # launches bracketed by HIP events (direct launches while timing)
    labs = synth.target_labels(pb, 16, seed=1)
    per_class = {}
    for k, name in BATCH_KNAMES.items():
        op.time_kernel(k, True)
        t0 = time.perf_counter()
        op.solve_batch(labs, pb.betas, rtol=SOLVE_RTOL, chunk=args.batch_chunk)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms, nl = op.kernel_time()
        op.time_kernel(k, False)
        per_class[name] = {"ms": round(ms, 1), "launches": nl, "us_per_launch": round(1e3 * ms / max(nl, 1), 1),
                           "solve_s": round(dt, 2)}
        log("  %-10s %8.1f ms %6d launches %9.1f us/launch (solve %.2f s)"
            % (name, ms, nl, 1e3 * ms / max(nl, 1), dt))
    op.close()
    print(json.dumps({"experiment": "batched-targets", "workload": pb.name, "rtol": pb.rtol, "autotune": tune,
                      "rows": rows, "many_targets": many, "per_kernel_16_targets": per_class}))


def shifted_table(args, fsda, torch):
    """CG per shift versus the shared-basis recurrence on (X^T X + beta I) w = X^T z, tolerance 1e-3."""
    import synth
    t0 = time.perf_counter()
    pb = synth.workload("chembl", seed=args.seed, cache_dir=args.cache)
    log("chembl-shaped matrix in %.1fs: %s" % (time.perf_counter() - t0, pb.summary()))
    op = fsda.Operator.from_problem(pb, max_shifts=12, max_chunk=args.chunk)
    z = op.sa_rhs()  # the centred labels y_c as the regressed sample-space vector
    rows = []
    for betas, p_cg, p_sh, p_sp in SHIFTED_TABLE:
        res = {}
        for shared in (True, False):
            op.regression_solve(z, betas, rtol=pb.rtol, chunk=args.chunk, shared_basis=shared)  # warm
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            W, it, rel, st = op.regression_solve(z, betas, rtol=pb.rtol, chunk=args.chunk, shared_basis=shared)
            torch.cuda.synchronize()
            res[shared] = (time.perf_counter() - t1, it, rel, st)
        cg_s, sh_s = res[False][0], res[True][0]
        rows.append({"betas": list(betas), "cg_s": round(cg_s, 4), "shifted_s": round(sh_s, 4),
                     "speedup": round(cg_s / sh_s, 3), "iters_cg": res[False][1].tolist(),
                     "iters_shifted": res[True][1].tolist(),
                     "worst_relres": max(float(res[False][2].max()), float(res[True][2].max())),
                     "paper": {"cg_s": p_cg, "shifted_s": p_sh, "speedup": p_sp}})
        log("table row: CG %.3fs shifted %.3fs speed-up %.2f (paper %.2f)" % (cg_s, sh_s, cg_s / sh_s, p_sp))
    print(json.dumps({"experiment": "shifted-table", "unit": "s", "tolerance": pb.rtol,
                      "workload": "chembl-shaped: n=%d x d=%d binary, nnz_X=%d, Zipf %.1f feature popularity; "
                                  "regressed vector y_c of %d labeled rows"
                                  % (pb.n, pb.d, pb.x_nnz, 1.1, pb.lab_idx.size),
                      "rows": rows}), flush=True)


def _rocpd_tables(d: str, pattern: str):
    """(kernel stats, per-dispatch counters) as pandas frames from rocprofv3 output in directory d:
    its SQLite database (*_results.db, the default format) or its CSV files."""
    import glob
    import sqlite3
    import pandas as pd
    stats, counters = [], []
    for f in sorted(glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True)):
        c = sqlite3.connect(f)
        stats.append(pd.read_sql_query("select name as Name, total_calls as Calls, total_duration as TotalDurationNs, "
                                       "average as AverageNs, percentage as Percentage from top_kernels", c))
        counters.append(pd.read_sql_query("select kernel_name as Kernel_Name, counter_name as Counter_Name, "
                                          "value as Counter_Value from counters_collection", c))
        c.close()
    for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
        stats.append(pd.read_csv(f))
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        counters.append(pd.read_csv(f))
    cat = lambda fs: pd.concat(fs, ignore_index=True) if fs else None  # noqa: E731
    return cat(stats), cat(counters)


def summarize_rocprof(d: str, kernel_substr: str, calib_mib: int) -> str:
    """Condenses rocprofv3 output in directory d into a few lines of text: the
    kernel statistics (durations) and the per-dispatch counters averaged per kernel
    (first 90 characters of the name); for the calibration copy the dispatches whose
    count is at least half of the largest are averaged (the plain copy of calib_mib MiB)."""
    lines = []
    stats, counters = _rocpd_tables(d, "")
    if stats is not None and len(stats):
        stats["Name"] = stats["Name"].str.slice(0, 90)
        lines.append("kernel statistics (durations in ns):")
        lines.append(stats[["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"]].head(20).to_string())
    if counters is not None and len(counters):
        counters["Kernel_Name"] = counters["Kernel_Name"].str.slice(0, 90)
        for cname, g in counters.groupby("Counter_Name"):
            agg = g.groupby("Kernel_Name")["Counter_Value"].agg(["count", "mean"]).sort_values("mean",
                                                                                           ascending=False)
            lines.append("counter %s (mean per dispatch):" % cname)
            sel = agg[[kernel_substr in k or "copy" in k.lower() for k in agg.index]]
            lines.append(sel.head(12).to_string())
            cp = g[g["Kernel_Name"].str.lower().str.contains("copy")]
            if len(cp) and calib_mib > 0:
                big = cp[cp["Counter_Value"] >= 0.5 * cp["Counter_Value"].max()]
                lines.append("calibration copy of %d MiB: %s = %.1f KiB per dispatch over %d dispatches"
                             % (calib_mib, cname, big["Counter_Value"].mean(), len(big)))
    return "\n".join(lines)


TRAFFIC_MATCH = {"k_xt": "k_xt<fsda::EpiXTR<double>", "k_xt_lds": "k_xt_lds<double>",
                 "k_rows_x": "k_rows<fsda::EpiX<double, false>, 1024>", "k_fold": "k_fold_apply<double>",
                 "k_rows_s": "k_rows<fsda::EpiLap<double, false>", "k_assemble": "k_assemble<fsda::EpiXTR<double>"}


def traffic_lines(dfetch: str, dwrite: str, calib_mib: int, workload: str) -> str:
    """TRAFFIC lines (HBM bytes per launch) from a FETCH_SIZE run and a WRITE_SIZE run.

    Each counter is calibrated on the plain device copy of calib_mib MiB recorded in
    the same run (its per-dispatch value against the bytes it must read or write)."""
    sha = kernel_source_key()
    per = {}
    for d, cname in ((dfetch, "FETCH_SIZE"), (dwrite, "WRITE_SIZE")):
        _, df = _rocpd_tables(d, "")
        g = df[df["Counter_Name"] == cname]
        cp = g[g["Kernel_Name"].str.lower().str.contains("copy")]
        big = cp[cp["Counter_Value"] >= 0.5 * cp["Counter_Value"].max()]
        factor = (calib_mib << 20) / (big["Counter_Value"].mean() * 1024.0)
        out = {"factor": factor}
        for key, sub in TRAFFIC_MATCH.items():
            sel = g[g["Kernel_Name"].str.contains(sub, regex=False)]
            if len(sel):
                out[key] = (float(sel["Counter_Value"].mean()), len(sel))
        per[cname] = out
    lines = ["calibration factors: FETCH_SIZE x %.4f, WRITE_SIZE x %.4f (KiB per dispatch -> bytes / 1024)"
             % (per["FETCH_SIZE"]["factor"], per["WRITE_SIZE"]["factor"])]
    for key in TRAFFIC_MATCH:
        if key in per["FETCH_SIZE"] and key in per["WRITE_SIZE"]:
            fk, fn = per["FETCH_SIZE"][key]
            wk, wn = per["WRITE_SIZE"][key]
            rb = fk * 1024 * per["FETCH_SIZE"]["factor"]
            wb = wk * 1024 * per["WRITE_SIZE"]["factor"]
            lines.append("TRAFFIC kernel=%s workload=%s source=%s bytes=%d read=%d written=%d dispatches=%d,%d"
                         % (key, workload, sha, rb + wb, rb, wb, fn, wn))
    return "\n".join(lines)


STEP_TARGETS = 64     # targets per step (one fsda_multishift_solve_batch call)
TOTAL_TARGETS = 1000  # the many-targets configuration; steps take the next 64, cyclically


def roofline_large(args, fsda, torch):
    """The operator apply on the large workload, whose vectors (p: 32 MB, t and u:
    12 MB) and index arrays (0.9 GB) are far beyond the 256 MB Infinity Cache.

    For each apply kernel class, one solve limited to `roof_iters` iterations
    runs with HIP events around every launch of that class (on the launch
    stream); average launch time = event time / launches (a pair costs a few
    microseconds, under 2 % of these kernels; it is not subtracted).  The
    dominant kernel's algorithmic bytes over its average time give `achieved`;
    the operator apply is B_op = 8Z + 4G + 40N + 28D over the summed averages.
    Also the time of one shared iteration over all 32 shifts (difference of
    two solves of m and 2m iterations, graph replay) and the oracle's time per
    per-shift CG iteration on the host, extrapolated."""
    import synth
    t0 = time.perf_counter()
    pb = synth.workload("large", seed=args.seed, cache_dir=args.cache)
    log("large workload in %.1fs: %s" % (time.perf_counter() - t0, pb.summary()))
    op = fsda.Operator.from_problem(pb, max_chunk=128)
    S = pb.betas.size
    m = args.roof_iters
    op.solve(pb.betas, rtol=pb.rtol, maxit=m, chunk=128)  # warm (graph capture)
    torch.cuda.synchronize()
    per = {}
    for k in APPLY_CLASSES:
        op.time_kernel(k, True, every=1)
        op.solve(pb.betas, rtol=pb.rtol, maxit=m, chunk=128)
        ms, nl = op.kernel_time()
        op.time_kernel(k, False)
        if nl:
            per[k] = (ms, nl)
            log("large: %-40s %8.1f us per launch over %d launches" % (KNAMES[k], 1e3 * ms / nl, nl))
    # one shared iteration (all shifts), from solves of m and 2m iterations
    sec = []
    for mm in (m, 2 * m):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        W, it, rel, st = op.solve(pb.betas, rtol=pb.rtol, maxit=mm, chunk=128)
        torch.cuda.synchronize()
        sec.append(time.perf_counter() - t1)
        del W
    iter_s = (sec[1] - sec[0]) / m
    pair_us = event_pair_us(torch)
    op.close()
    del op
    copy_gbs = copy_ceiling(torch)
    dom = max(per, key=lambda k: per[k][0] / per[k][1])
    ms, nl = per[dom]
    avg_us = 1e3 * ms / nl
    bytes_launch = algorithmic_bytes(dom, pb, S, 128)
    achieved = bytes_launch / (avg_us * 1e-6) / 1e9
    apply_us = sum(1e3 * v[0] / v[1] for v in per.values())
    b_op = 8 * pb.x_nnz + 4 * pb.s_nnz + 40 * pb.n + 28 * pb.d
    roof = {"bound": "hbm", "workload": "large: n=%d x d=%d, nnz_X=%d, nnz_S=%d" % (pb.n, pb.d, pb.x_nnz, pb.s_nnz),
            "kernel": KNAMES[dom], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom, "large"),
            "bytes_per_launch": bytes_launch, "avg_launch_us": round(avg_us, 2), "launches": nl,
            "timed_every": 1, "event_pair_us": round(pair_us, 2), "xt_plan": xt_plan(pb)["plan"],
            "note": "HIP events around every launch of the kernel on its launch stream, pair cost included",
            "copy_ceiling_GBps": round(copy_gbs, 1), "frac_of_copy_ceiling": round(achieved / copy_gbs, 4),
            "traffic_note": "rocprofv3 FETCH_SIZE + WRITE_SIZE (beyond L2: Infinity Cache or HBM) per launch, "
                            "calibrated on a 1 GiB device copy in the same run; a lower bound (the counters "
                            "read 0.26 to 0.43 of the fold's 12.3 GB pure stream), see profiles/large_apply_traffic.txt"}
    apply = {"workload": "large", "bytes": b_op, "us": round(apply_us, 2),
             "GBps": round(b_op / (apply_us * 1e-6) / 1e9, 1),
             "frac": round(b_op / (apply_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
             "frac_of_copy_ceiling": round(b_op / (apply_us * 1e-6) / 1e9 / copy_gbs, 4),
             "kernels_us": {KNAMES[k]: round(1e3 * v[0] / v[1], 2) for k, v in per.items()},
             "note": "X, graph and X^T kernels of one iteration (the X^T pass also updates r, bytes not counted)"}
    gpu_iter = {"seconds_per_shared_iteration": round(iter_s, 6), "shifts": S,
                "note": "one iteration of the shared recurrence for all %d shifts, fold included, graph replay" % S}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t1 = time.perf_counter()
        oracle.solve(pb, betas=[pb.betas[-1]], rtol=pb.rtol, maxit=1)
        one = time.perf_counter() - t1
        t1 = time.perf_counter()
        oracle.solve(pb, betas=[pb.betas[-1]], rtol=pb.rtol, maxit=3)
        three = time.perf_counter() - t1
        cpu = {"seconds_per_iteration": round((three - one) / 2, 4), "cores": oracle.max_threads(),
               "kind": "oracle", "note": "per-shift FP64 CG of the oracle on the large workload, one iteration of "
                                         "one shift (difference of 3- and 1-iteration solves), extrapolated: a "
                                         "per-shift CG needs one such iteration per shift per step of its own"}
        log("large: oracle %.3f s per iteration on %d threads" % (cpu["seconds_per_iteration"], cpu["cores"]))
    return roof, apply, gpu_iter, cpu


def cpu_baseline_targets(pb, target, budget_s: float, rtol: float):
    """The oracle (per-shift FP64 CG) on the host cores for one target of the
    many-targets workload: its largest and smallest shift, then a 1-thread run of
    a few iterations of the largest, extrapolated to the same iteration counts."""
    import dataclasses
    import oracle
    pc = dataclasses.replace(pb, lab_idx=target[0], lab_y=target[1])
    nt = oracle.max_threads()
    solved, spent, sample, iters = 0, 0.0, [], 0
    for s in (int(np.argmax(pb.betas)), int(np.argmin(pb.betas))):
        if spent > budget_s:
            break
        t0 = time.perf_counter()
        W, it, rel, rc = oracle.solve(pc, betas=[pb.betas[s]], rtol=rtol, maxit=20000)
        dt = time.perf_counter() - t0
        spent += dt
        iters += int(it[0])
        solved += bool(rel[0] <= TARGET_RELRES)
        sample.append({"beta": float(pb.betas[s]), "iters": int(it[0]), "seconds": round(dt, 3),
                       "relres": float(rel[0])})
    one_core = None
    try:
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oracle.solve(pc, betas=[pb.betas[-1]], rtol=rtol, maxit=2)
        t2 = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.solve(pc, betas=[pb.betas[-1]], rtol=rtol, maxit=12)
        t12 = time.perf_counter() - t0
        per_it = (t12 - t2) / 10
        one_core = {"value": round(solved / (per_it * iters), 5) if iters else 0.0, "unit": "solves/s", "cores": 1,
                    "seconds_per_iteration": round(per_it, 4),
                    "note": "extrapolated: 1-thread time per iteration x the iterations of the sample above"}
    finally:
        oracle.set_threads(nt)
    return {"value": solved / spent if spent > 0 else 0.0, "unit": "solves/s", "cores": nt, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cores": host_cores(),
            "sample": "per-shift FP64 CG of the oracle for target 0 of the first timed step (its own labeled set "
                      "of %d rows) on the same mid-scale X and graph, for 2 of its %d shifts (largest and smallest "
                      "beta) to rel. residual %.0e: %s" % (target[0].size, pb.betas.size, rtol, json.dumps(sample)),
            "one_core": one_core}


def cpu_baseline_diff(pb, target, iters_total: int, nhyper: int):
    """The oracle on the host cores for the differentiation workload, extrapolated:
    the time of one per-shift FP64 CG iteration with one target's training labels
    (difference of a 12- and a 2-iteration solve), all threads and one thread, times
    the iterations the GPU needed for every forward and adjoint system (a per-shift
    CG needs about as many for its shift as the shared recurrence took to meet it)."""
    import dataclasses
    import oracle
    pc = dataclasses.replace(pb, lab_idx=target[0], lab_y=target[1])
    nt = oracle.max_threads()

    def per_iteration():
        t0 = time.perf_counter()
        oracle.solve(pc, betas=[pb.betas[-1]], rtol=pb.rtol, maxit=2)
        t2 = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.solve(pc, betas=[pb.betas[-1]], rtol=pb.rtol, maxit=12)
        return (time.perf_counter() - t0 - t2) / 10

    per_it = per_iteration()
    try:
        oracle.set_threads(1)
        per_it1 = per_iteration()
    finally:
        oracle.set_threads(nt)
    return {"value": round(nhyper / (per_it * iters_total), 5), "unit": "hypergradients/s", "cores": nt,
            "kind": "oracle", "cpu_model": cpu_model(), "host_cores": host_cores(),
            "sample": "extrapolated: %.4f s per per-shift FP64 CG iteration of the oracle (target 0's training "
                      "labels, difference of 12- and 2-iteration solves) x %d iterations (the GPU's iteration "
                      "counts of all 64 x %d forward and adjoint systems)" % (per_it, iters_total, pb.betas.size),
            "one_core": {"value": round(nhyper / (per_it1 * iters_total), 6), "unit": "hypergradients/s",
                         "cores": 1, "seconds_per_iteration": round(per_it1, 4)}}


def batched_bench(args, fsda, torch):
    """The default benchmark: shifted solves per second of many targets over one X."""
    import synth
    t0 = time.perf_counter()
    pb = synth.workload("mid", seed=args.seed, cache_dir=args.cache)
    log("mid workload in %.1fs: %s" % (time.perf_counter() - t0, pb.summary()))
    t0 = time.perf_counter()
    targets = synth.target_labels(pb, TOTAL_TARGETS, seed=2)
    labeled = np.array([t[0].size for t in targets])
    log("%d targets in %.1fs (labeled rows: median %d, min %d, max %d)"
        % (len(targets), time.perf_counter() - t0, np.median(labeled), labeled.min(), labeled.max()))
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    op = fsda.Operator.from_problem(pb, max_chunk=128)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    tile, groups, rates = op.autotune_batch(targets[:16], pb.betas, trial_iters=32)
    tune = {"tile": tile, "groups_per_row": groups, "seconds": round(time.perf_counter() - t0, 2),
            "shifted_target_iterations_per_s": {"%dx%d" % sh: round(r, 1) for sh, r in rates.items()}}
    log("autotuned tile %d, %d groups per row: %s" % (tile, groups, tune["shifted_target_iterations_per_s"]))
    S = pb.betas.size
    group = [0]

    def step():
        k = group[0]
        group[0] += 1
        labs = [targets[(k * STEP_TARGETS + j) % TOTAL_TARGETS] for j in range(STEP_TARGETS)]
        W, iters, relres, st = op.solve_batch(labs, pb.betas, rtol=SOLVE_RTOL, chunk=args.batch_chunk)
        del W
        return iters, relres, st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    first_timed = group[0]
    log("warmup done")
    t0 = time.perf_counter()
    solved, worst, maxit, statuses = 0, 0.0, 0, set()
    for _ in range(args.steps):
        iters, relres, st = step()
        solved += int((relres <= TARGET_RELRES).sum())
        worst = max(worst, float(relres.max()))
        maxit = max(maxit, int(iters.max()))
        statuses.add(int(st))
        log("step done: %d of %d solved so far" % (solved, STEP_TARGETS * S * (group[0] - first_timed)))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = solved / elapsed
    # the plain per-target FP64 path on the same X: the mid workload's own labeled set
    op.solve(pb.betas, rtol=SOLVE_RTOL, chunk=128)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    psolved = 0
    for _ in range(3):
        W, it1, rel1, st1 = op.solve(pb.betas, rtol=SOLVE_RTOL, chunk=128)
        psolved += int((rel1 <= TARGET_RELRES).sum())
        del W
    torch.cuda.synchronize()
    per_target = psolved / (time.perf_counter() - t0)
    log("batched %.2f shifted solves/s; per-target FP64 path %.2f solves/s" % (value, per_target))
    op.close()
    del op
    roof, apply, gpu_iter, cpu_large = roofline_large(args, fsda, torch)
    out = {
        "metric": "shifted SDA solves/sec at rel. residual 1e-8",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched targets: %d binary targets per step (of %d, labeled fraction lognormal "
                               "around 0.7%% in [0.1%%, 5%%], positive rate U(2%%, 30%%)) x %d shifts logspace(-3, 2) "
                               "over X n=%d x d=%d binary (nnz_X=%d, Zipf 1.1) and a 10-NN graph (nnz_S=%d), "
                               "alpha=%g, rtol %g, FP64" % (STEP_TARGETS, TOTAL_TARGETS, S, pb.n, pb.d, pb.x_nnz,
                                                          pb.s_nnz, pb.alpha, pb.rtol),
                   "graph": graph_stats(pb),
                   "targets_per_step": STEP_TARGETS, "total_targets": TOTAL_TARGETS, "shifts": S, "n": pb.n,
                   "d": pb.d, "nnz_x": pb.x_nnz, "nnz_s": pb.s_nnz, "tile": tile, "groups_per_row": groups},
        "roofline": roof,
        "operator_apply": apply,
        "detail": {"per_target_fp64_solves_per_s": round(per_target, 3),
                   "speedup_vs_per_target_fp64": round(value / per_target, 3) if per_target > 0 else None,
                   "per_target_fp64_iters": it1.tolist(), "worst_relres": worst, "max_iters": maxit,
                   "solver_rtol": SOLVE_RTOL, "counted_at": TARGET_RELRES, "statuses": sorted(statuses), "solved": solved, "solves_attempted": args.steps * STEP_TARGETS * S,
                   "targets_timed": [first_timed * STEP_TARGETS % TOTAL_TARGETS, group[0] * STEP_TARGETS],
                   "build_s": round(build_s, 3), "autotune": tune, "large_iteration": gpu_iter,
                   "cpu_large": cpu_large},
    }
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline_targets(pb, targets[(first_timed * STEP_TARGETS) % TOTAL_TARGETS],
                                                   args.cpu_budget, pb.rtol)
        log("cpu baseline took %.1fs" % (time.perf_counter() - t0))
    print(json.dumps(out), flush=True)


def diff_experiment(args, fsda, torch):
    """The differentiation workload (500,000 x 2,000,000, about 60 nonzeros per row,
    alpha 0.9, 8 shifts logspace(-3, 2)): 64 targets (labeled sets as in the
    many-targets workload), each split 80/20 into training labels and held-out rows.
    Times the phases of the hypergradient: the forward solves of every target
    (fsda_multishift_solve_batch), the hold-out losses and adjoint right-hand sides
    (fsda_holdout_batch), the 64 x 8 adjoint systems (fsda_solve_columns_batch, asked
    for half of rtol on its recursive residual so that the true residuals meet rtol)
    and the gradient in (log beta, alpha) (fsda_hypergradient_batch); reports the
    library's own true residuals.  (The oracle's recomputation of sampled residuals
    and gradients at this size is tests/test_gpu_diff.py.)"""
    import synth
    t0 = time.perf_counter()
    pb = synth.workload("diff", seed=args.seed, cache_dir=args.cache)
    log("diff workload in %.1fs: %s" % (time.perf_counter() - t0, pb.summary()))
    train, held = synth.holdout_splits(synth.target_labels(pb, 64, seed=5), seed=5)
    op = fsda.Operator.from_problem(pb, max_chunk=128)
    S = pb.betas.size
    op.solve_batch(train[:16], pb.betas, rtol=pb.rtol)  # warm (graph capture, kernels)
    phases = {}

    def timed(name, fn):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        phases[name] = round(time.perf_counter() - t1, 3)
        log("%s: %.2f s" % (name, phases[name]))
        return r

    W, it, rel, st = timed("forward_s", lambda: op.solve_batch(train, pb.betas, rtol=pb.rtol))
    loss, G = timed("holdout_s", lambda: op.holdout_batch(W, held))

    # in groups of ADJ targets, a line after each: the library takes a call's columns
    # shift by shift in tiles of 16, so with 16 targets per call every tile holds one
    # shift (similar iteration counts), where 8 per call pair neighbouring shifts
    ADJ = 16

    def adjoint():
        Lam = torch.empty_like(G)
        its = np.zeros((64, S), dtype=np.int32)
        rels = np.zeros((64, S))
        worst = fsda.OK
        for c0 in range(0, 64, ADJ):
            L, i2, r2, s2 = op.solve_columns_batch(train[c0:c0 + ADJ], pb.betas, G[c0:c0 + ADJ],
                                                   rtol=0.5 * pb.rtol)
            Lam[c0:c0 + ADJ], its[c0:c0 + ADJ], rels[c0:c0 + ADJ] = L, i2, r2
            worst = max(worst, s2)
            log("adjoint targets %d..%d done" % (c0, c0 + ADJ - 1))
        return Lam, its, rels, worst

    Lam, it2, rel2, st2 = timed("adjoint_s", adjoint)
    dlb, da = timed("gradient_s", lambda: op.hypergradient_batch(train, W, Lam, pb.betas))
    total = sum(phases.values())
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_diff(pb, train[0], int(it.sum()) + int(it2.sum()), 64 * S)
        log("cpu baseline: %s" % json.dumps(cpu))
    print(json.dumps({"experiment": "diff", "workload": "diff: n=%d x d=%d binary, nnz_X=%d, nnz_S=%d, alpha=%g, "
                                                        "%d shifts, 64 targets (80/20 splits), rtol %g"
                                                        % (pb.n, pb.d, pb.x_nnz, pb.s_nnz, pb.alpha, S, pb.rtol),
                      "phases_s": phases, "total_s": round(total, 3),
                      "hypergradients_per_s": round(64 * S / total, 2),
                      "forward": {"status": st, "worst_relres": float(rel.max()), "max_iters": int(it.max()),
                                  "solved": int((rel <= TARGET_RELRES).sum())},
                      "adjoint": {"status": st2, "worst_relres": float(rel2.max()), "max_iters": int(it2.max()),
                                  "solved": int((rel2 <= TARGET_RELRES).sum()), "iters_sum": int(it2.sum()),
                                  "targets_per_call": ADJ},
                      "finite": bool(np.isfinite(dlb).all() and np.isfinite(da).all()),
                      "loss_range": [float(loss.min()), float(loss.max())], "cpu_baseline": cpu}), flush=True)


def mixed_large(args, fsda, torch):
    """The whole shift grid of the large workload solved in FP64 and by the mixed
    path (FP32 shared recurrence, one FP64 refinement step), each timed once from
    the right-hand side to the reported true residuals, with the mixed path's
    iterations per shift."""
    import synth
    os.environ.setdefault("FSDA_PROGRESS", "20")  # the solve loops print their iteration count
    pb = synth.workload("large", seed=args.seed, cache_dir=args.cache, log=log)
    torch.cuda.set_device(0)
    S = pb.betas.size
    out = {}
    for name, prec in (("fp64", fsda.FP64), ("mixed", fsda.MIXED)):
        op = fsda.Operator.from_problem(pb, precision=prec, max_chunk=128)
        W = torch.empty((S, pb.d), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        log("%s: solving %d shifts" % (name, S))
        t0 = time.perf_counter()
        b = op.rhs()
        _, iters, relres, st = op.solve(pb.betas, rtol=pb.rtol, chunk=128, b=b, out=W)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        rep = op.solve_report(S)
        ok = int((relres <= pb.rtol).sum())
        out[name] = {"seconds": round(sec, 2), "status": int(st), "shifts_within_rtol": ok,
                     "worst_relres": float(relres.max()), "relres": [float("%.3e" % r) for r in relres],
                     "iters": [int(i) for i in iters], "main_iters": [int(i) for i in rep["main_iters"]],
                     "refine_iters": [int(i) for i in rep["refine_iters"]],
                     "refine_steps": [int(i) for i in rep["steps"]]}
        log("%s: %.2f s, status %d, %d of %d shifts within rtol, worst relres %.3e, max main iterations %d, "
            "max correction iterations %d" % (name, sec, st, ok, S, relres.max(), rep["main_iters"].max(),
                                               rep["refine_iters"].max()))
        op.close()
        del W
    print(json.dumps({"experiment": "mixed-large", "workload": "large: n=%d x d=%d, nnz_X=%d, nnz_S=%d, %d shifts "
                      "%.0e..%.0e, rtol %.0e" % (pb.n, pb.d, pb.x_nnz, pb.s_nnz, S, pb.betas.min(), pb.betas.max(),
                                                  pb.rtol), **out}), flush=True)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-rocprof":
        # python bench.py --summarize-rocprof DIR KERNEL_SUBSTR CALIB_MIB
        print(summarize_rocprof(sys.argv[2], sys.argv[3], int(sys.argv[4])))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--traffic-lines":
        # python bench.py --traffic-lines FETCH_DIR WRITE_DIR CALIB_MIB WORKLOAD
        print(traffic_lines(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5]))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 8 batched, 10 single-target)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (default 1 batched, 2 single)")
    ap.add_argument("--workload", default="batched",
                    help="'batched' (default): many targets over the mid-scale X, roofline on large; or one "
                         "workload's single-target path: mid, large, tiny, diff")
    ap.add_argument("--roof-iters", type=int, default=128,
                    help="iterations per timed solve of the large-workload roofline (one launch per class each)")
    ap.add_argument("--chunk", type=int, default=128)
    ap.add_argument("--batch-chunk", type=int, default=0,
                    help="fold interval of the target batches (0: the library's default)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=25.0)
    ap.add_argument("--cache", default=os.path.join(ROOT, ".synth_cache"))
    ap.add_argument("--kernel", type=int, default=-1,
                    help="kernel class to time in the timed region (default: the one with the largest total time)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (profiler calibration of byte counters)")
    ap.add_argument("--event-every", type=int, default=7,
                    help="in the timed region, HIP events around every N-th launch of the timed kernel class "
                         "(each pair costs a few microseconds of stream time; N prime to the fold interval, so "
                         "the samples visit every position in a chunk)")
    ap.add_argument("--graph-steps", type=int, default=2,
                    help="extra timed steps with kernel timing off (chunks replayed as HIP graphs), reported in detail")
    ap.add_argument("--no-paths", action="store_true", help="skip timing the further entry points (detail.paths)")
    ap.add_argument("--no-gather-ceiling", action="store_true",
                    help="skip timing the bare gathers of the dominant product's index stream")
    ap.add_argument("--targets", type=int, default=0,
                    help="batched-targets experiment: also solve this many targets, in calls of 64")
    ap.add_argument("--experiment", default="",
                    help="'shifted-table': the CG versus shifted CG table instead; 'gather-ceiling': the rate of "
                         "random gathers the sparse products are bound by; 'batched-targets': 16, 32 and 64 targets; "
                         "'roofline-large': the operator-apply roofline on the large workload alone; 'diff': the "
                         "hypergradient of 64 targets on the differentiation workload; 'mixed-large': the large "
                         "workload's whole shift grid in FP64 and by the mixed path")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1709_04794_amd as fsda

    if args.experiment and args.workload == "batched":
        args.workload = "mid"  # the experiments run on one workload's X
    if args.experiment == "shifted-table":
        shifted_table(args, fsda, torch)
        return
    if args.experiment == "gather-ceiling":
        gather_ceiling(args, fsda, torch)
        return
    if args.experiment == "batched-targets":
        batched_targets(args, fsda, torch)
        return
    if args.experiment == "diff":
        diff_experiment(args, fsda, torch)
        return
    if args.experiment == "mixed-large":
        mixed_large(args, fsda, torch)
        return
    if args.experiment == "roofline-large":
        if args.calib_copy_mb > 0:
            calibration_copy(torch, args.calib_copy_mb)
        roof, apply, gpu_iter, cpu_large = roofline_large(args, fsda, torch)
        print(json.dumps({"experiment": "roofline-large", "roofline": roof, "operator_apply": apply,
                          "large_iteration": gpu_iter, "cpu_large": cpu_large}), flush=True)
        return
    if args.experiment:
        print("unknown experiment %r" % args.experiment, file=sys.stderr)
        sys.exit(2)

    batched = args.workload == "batched"
    if args.steps is None:
        args.steps = 8 if batched else 10
    if args.warmup is None:
        args.warmup = 1 if batched else 2
    if batched:
        batched_bench(args, fsda, torch)
        return
    single_bench(args, fsda, torch)


def copy_ceiling(torch, mib: int = 2048, reps: int = 5) -> float:
    """A measured stream ceiling of this GPU: GB/s of a plain device copy of `mib`
    MiB (read + write counted), the median of `reps` copies timed with events."""
    a = torch.empty((mib << 20) // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    c = torch.empty_like(a)
    c.copy_(a)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        c.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del a, c
    torch.cuda.empty_cache()
    return 2 * (mib << 20) / float(np.median(ts)) / 1e9


def calibration_copy(torch, mib: int):
    """A plain device copy of `mib` MiB, three times (the reference of the profiler's byte counters)."""
    nb = mib << 20
    a = torch.empty(nb // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    log("calibration copy: %d MiB read + %d MiB written per launch, 3 launches" % (mib, mib))


def single_bench(args, fsda, torch):
    """The single-target path of one workload: a step is the right-hand side, the
    multi-shift solve of every shift with the FP64 true-residual check, and the
    ratings s = X w."""
    import synth
    if args.calib_copy_mb > 0:
        calibration_copy(torch, args.calib_copy_mb)

    t0 = time.perf_counter()
    pb = synth.workload(args.workload, seed=args.seed, cache_dir=args.cache)
    log("workload %s generated in %.1fs: %s" % (args.workload, time.perf_counter() - t0, pb.summary()))
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    op = fsda.Operator.from_problem(pb, max_chunk=max(args.chunk, 1))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log("operator built in %.2fs (workspace %.1f MB)" % (build_s, op.ws_bytes / 1e6))
    S = pb.betas.size
    W = torch.empty((S, pb.d), dtype=torch.float64, device="cuda")

    def step():
        b = op.rhs()
        Wt, iters, relres, st = op.solve(pb.betas, rtol=pb.rtol, chunk=args.chunk, b=b, out=W)
        op.project(Wt)
        return iters, relres, st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")

    # which kernel dominates: one pass per kernel class with that class timed
    per_class = {}
    if args.kernel < 0:
        for k in KNAMES:
            op.time_kernel(k, True)
            step()
            ms, nl = op.kernel_time()
            per_class[k] = (ms, nl)
            op.time_kernel(k, False)
            log("class %s timed: %.3f ms per step" % (KNAMES[k], ms))
        dom = max(per_class, key=lambda k: per_class[k][0])
        log("per-kernel ms per step: %s" % {KNAMES[k]: round(v[0], 3) for k, v in per_class.items()})
    else:
        dom = args.kernel

    op.time_kernel(dom, True, every=args.event_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solved = 0
    worst = 0.0
    iters_seen = None
    for _ in range(args.steps):
        iters, relres, st = step()
        solved += int((relres <= TARGET_RELRES).sum())
        worst = max(worst, float(relres.max()))
        iters_seen = iters
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kms, klaunch = op.kernel_time()
    op.time_kernel(dom, False)

    graph_rate = None
    if args.graph_steps > 0:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gsolved = 0
        for _ in range(args.graph_steps):
            iters_g, relres_g, _ = step()
            gsolved += int((relres_g <= TARGET_RELRES).sum())
        torch.cuda.synchronize()
        graph_rate = gsolved / (time.perf_counter() - t1)
        log("graph-replay steps: %.3f solves/s" % graph_rate)

    # the event pair around each timed launch costs some time of its own on the
    # stream: measure empty pairs the same way and take that off
    pair_us = event_pair_us(torch)
    raw_launch_s = (kms / 1e3) / max(klaunch, 1)
    avg_launch_s = max(raw_launch_s - pair_us * 1e-6, 1e-9)
    # the operator apply of one iteration (X, graph and X^T passes) against its
    # algorithmic bytes 8Z + 4G + 40N + 28D (index arrays once, vectors once);
    # the residual update fused into the X^T pass rides along uncounted, and the
    # long rows of X^T are finished in the direction update, outside this time
    op_apply = None
    if per_class:
        us = 0.0
        for k in (fsda.K_X, fsda.K_S, fsda.K_XT, fsda.K_XTL, fsda.K_RESID):
            ms, nl = per_class.get(k, (0.0, 0))
            if nl:
                us += max(1e3 * ms / nl - pair_us, 0.0)
        b_op = 8 * pb.x_nnz + 4 * pb.s_nnz + 40 * pb.n + 28 * pb.d
        op_apply = {"bytes": b_op, "us": round(us, 2), "GBps": round(b_op / (us * 1e-6) / 1e9, 1),
                    "frac": round(b_op / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                    "note": "X, graph and X^T passes of one iteration (the X^T pass also updates r, bytes not "
                            "counted; with LDS slices it is two kernels, both counted); HIP-event times minus "
                            "the event-pair overhead"}
    bytes_launch = algorithmic_bytes(dom, pb, S, args.chunk)
    achieved = bytes_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    # the products are bound by random 8-byte gathers: time a bare gather kernel
    # on the dominant product's own index stream
    gather = None
    pname = {fsda.K_XT: "xt_short" if xt_plan(pb)["plan"] == "lds" else "xt", fsda.K_X: "x_cold",
             fsda.K_S: "s"}.get(dom)
    if pname is not None and not args.no_gather_ceiling:
        _, idx, size = gather_patterns(pb)[pname]
        g_us = time_gathers(fsda, torch, size, idx, pair_us=pair_us)
        gather = {"pattern": pname, "gathers": int(idx.size), "bare_gather_us": round(g_us, 2),
                  "kernel_us": round(avg_launch_s * 1e6, 2), "frac": round(g_us / (avg_launch_s * 1e6), 4),
                  "note": "time of a bare gather-and-add kernel over the same index stream / the kernel's "
                          "time (python bench.py --experiment gather-ceiling covers all three products)"}
    value = solved / elapsed
    ws_mb = (8 * pb.x_nnz + 4 * pb.s_nnz + 40 * pb.n + 28 * pb.d) / 1e6
    out = {
        "metric": "shifted SDA solves/sec at rel. residual 1e-8",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s: n=%d x d=%d binary, nnz_X=%d, kNN graph nnz_S=%d, l=%d labeled, alpha=%g, "
                               "%d shifts logspace, rtol %g" % (pb.name, pb.n, pb.d, pb.x_nnz, pb.s_nnz,
                                                                pb.lab_idx.size, pb.alpha, S, pb.rtol),
                   "n": pb.n, "d": pb.d, "nnz_x": pb.x_nnz, "nnz_s": pb.s_nnz, "shifts": S, "chunk": args.chunk,
                   "precision": "fp64"},
        "roofline": {"bound": "hbm", "workload": pb.name,
                     "memory": ("working set of one iteration %.0f MB fits the 256 MB Infinity Cache: these are cache "
                                "rates, not HBM rates" % (ws_mb,)) if ws_mb < 256 else "HBM (working set %.0f MB)" % ws_mb,
                     "kernel": KNAMES[dom], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom, args.workload),
                     "bytes_per_launch": bytes_launch, "avg_launch_us": round(avg_launch_s * 1e6, 2),
                     "launches": klaunch, "timed_every": args.event_every, "event_pair_us": round(pair_us, 2),
                     "avg_launch_us_with_events": round(raw_launch_s * 1e6, 2), "gather_ceiling": gather},
        "operator_apply": op_apply,
        "detail": {"iters": None if iters_seen is None else iters_seen.tolist(), "worst_relres": worst,
                   "solved_per_step": solved / args.steps, "build_s": round(build_s, 3),
                   "graph_replay_solves_per_s": graph_rate,
                   "per_kernel_ms_per_step": {KNAMES[k]: round(v[0], 3) for k, v in per_class.items()},
                   "per_kernel_launches_per_step": {KNAMES[k]: v[1] for k, v in per_class.items()}},
    }
    if not args.no_paths:
        t0 = time.perf_counter()
        op.close()
        del op
        out["detail"]["paths"] = time_paths(pb, fsda, torch, args.chunk)
        log("further entry points timed in %.1fs" % (time.perf_counter() - t0))
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(pb, args.cpu_budget)
        log("cpu baseline took %.1fs" % (time.perf_counter() - t0))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
