/*
 * fsda.h -- C ABI of the MI355X (gfx950) multi-shift solver for fast
 * semi-supervised discriminant analysis (FSDA; Tavernier et al., "Fast
 * semi-supervised discriminant analysis for binary classification of large
 * data-sets", arXiv:1709.04794).
 *
 * The library solves, for every regularisation value beta_s of a grid,
 *
 *     A(beta_s) w_s = b,   A(beta) = (X - 1 mu_l^T)^T [ (1-alpha) P_l + alpha L ] X + beta I_D
 *
 * (Alg. 7, step 4; the SDA eigenproblem of Eq. SDAeig centred on the labeled
 * mean as in Sec. 2.5.2 and Sec. 3.2.3), with one shared Krylov basis for all
 * shifts (Sec. 3.2.2, Alg. 3), and returns the ratings s_s = X w_s (Alg. 7,
 * return value).  Notation: X is the n x d binary sample-by-feature matrix,
 * l the number of labeled samples, mu_l = X^T 1_l / l the labeled mean,
 * P_l = diag(1_l) the labeled-sample selector, L = D - S the unnormalised
 * Laplacian of the binary similarity graph S (Sec. 2.3).
 *
 * Conventions for every entry point:
 *  - Pointers marked "device" are HIP device memory owned by the caller.  The
 *    library never allocates or frees device memory; all derived data lives in
 *    the caller's workspace.  Pointers marked "host" are ordinary host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on it; fsda_build_operator and fsda_multishift_solve return
 *    only after their work on `stream` has finished, the other calls return
 *    immediately after enqueueing.
 *  - Index arrays are int32: n, d and each nnz must be below 2^31.
 *  - A negative return value means nothing valid was written; the message is
 *    available from fsda_last_error() (per thread).  Arguments are validated
 *    on the host before any HIP call where that is possible.
 *  - One handle must not be used from two threads at once; distinct handles
 *    are independent.
 */
#ifndef FSDA_H
#define FSDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------- */
#define FSDA_OK 0             /* success                                              */
#define FSDA_NOT_CONVERGED 1  /* warning: some shift reached maxit; results valid     */
#define FSDA_E_ARG (-1)       /* bad argument (NULL pointer, size, handle)            */
#define FSDA_E_CSR (-2)       /* a CSR array is malformed (checked on the device)     */
#define FSDA_E_LABELS (-3)    /* labeled set invalid: out of range, repeated, one class */
#define FSDA_E_RANGE (-4)     /* alpha outside [0,1], beta <= 0, rtol <= 0, ...       */
#define FSDA_E_BREAKDOWN (-5) /* CG breakdown: <p, A p> <= 0 or not finite            */
#define FSDA_E_WORKSPACE (-6) /* workspace NULL, too small or misaligned              */
#define FSDA_E_HIP (-7)       /* a HIP runtime call failed                            */
#define FSDA_E_OVERFLOW (-8)  /* a size does not fit the int32 index type             */

/* ---- precision ------------------------------------------------------------- */
#define FSDA_FP64 0  /* every vector and scalar in FP64                              */
#define FSDA_MIXED 1 /* FP32 vectors and sparse products, FP64 dot products and     */
                     /* recurrence scalars, then FP64 refinement (see the solve)   */

/* Limits of one handle. */
#define FSDA_MAX_SHIFTS 64
#define FSDA_MAX_CHUNK 256
#define FSDA_MAX_TARGETS 4096   /* targets of one fsda_multishift_solve_batch call (in tiles) */
#define FSDA_MAX_COLUMNS 64     /* right-hand sides of one fsda_solve_columns call (one tile) */
#define FSDA_MAX_BATCH_CHUNK 128 /* fold interval of fsda_multishift_solve_batch */

typedef struct fsda_op fsda_op; /* opaque handle, host memory */

/*
 * The problem (Eq. SDAeig with the centring of Sec. 3.2.3):
 *  n, d            samples and features.
 *  x_rowptr[n+1], x_col[x_nnz]  (device) X in CSR form without values; every
 *                  stored entry is a 1 (binary fingerprints, Sec. 5.1).  Column
 *                  indices in [0, d), strictly increasing within a row.  The
 *                  library builds X^T itself, with the features relabeled by
 *                  decreasing frequency (an internal order; every vector the
 *                  caller sees is in the caller's feature order).
 *  s_rowptr[n+1], s_col[s_nnz]  (device) binary symmetric similarity S, no
 *                  self loops (Sec. 2.3-2.4); degree d_i = row length.  Symmetry
 *                  is the caller's responsibility (not checked).
 *  lab_idx[n_lab], lab_y[n_lab] (device) labeled samples (any order, no
 *                  repeats) and their classes +1 / -1.  Both classes present.
 *  alpha           weight of the manifold term, 0 <= alpha <= 1 (Eq. SDAeig).
 *  precision       FSDA_FP64 or FSDA_MIXED.
 * The handle borrows these arrays: they must stay valid and unchanged until
 * fsda_destroy_operator().
 */
typedef struct fsda_problem {
  int64_t n, d;
  const int32_t *x_rowptr, *x_col;
  int64_t x_nnz;
  const int32_t *s_rowptr, *s_col;
  int64_t s_nnz;
  const int32_t *lab_idx;
  const int8_t *lab_y;
  int64_t n_lab;
  double alpha;
  int precision;
} fsda_problem;

/*
 * Bytes of device workspace the handle needs for up to `max_shifts` shifts
 * (1..FSDA_MAX_SHIFTS) and a shift-state fold interval of up to `max_chunk`
 * iterations (1..FSDA_MAX_CHUNK; see fsda_multishift_solve).  Host only: no
 * HIP call.  *bytes (host) receives the size.
 */
int fsda_workspace_size(const fsda_problem *pb, int max_shifts, int max_chunk, size_t *bytes);

/*
 * Validates the problem, then builds the operator data in `workspace` (device,
 * 256-byte aligned, ws_bytes >= fsda_workspace_size()): the feature relabeling,
 * X and X^T in the internal order, the work partition of the three sparse
 * products, the labeled weights and the canonical right-hand side.  *out
 * (host) receives the handle.  Blocks until done.  The workspace belongs to the
 * handle until it is destroyed.
 * Plans of the X^T product (the longer rows of X^T are cut at sample
 * boundaries and their parts added in a fixed order):
 *  n <= 262,144: the rows of >= 64 nonzeros in LDS slices of 8192 samples;
 *    each work-group stages one slice of the sample-space vector in LDS and
 *    sums the rows' segments there.
 *  n > 262,144: the rows of >= 512 nonzeros in LDS slices, the rows of 16 to
 *    511 nonzeros in XCD slices: each of the eight XCDs gathers from one eighth
 *    of the sample range, which stays in its L2.
 * Results differ between plans only in the summation order of those rows.
 * The environment variable FSDA_XT_SLICES set to 1 (no slices), 8 (XCD slices
 * only), lds (LDS slices only, for n <= 262,144) or hyb (LDS and XCD slices)
 * overrides the choice, and FSDA_XT_HEAD the row length from which rows go to
 * LDS slices in the hybrid plan; they are read by fsda_workspace_size and by
 * this call, which must see the same values (else FSDA_E_WORKSPACE may result).
 * Errors: FSDA_E_ARG, FSDA_E_RANGE (alpha), FSDA_E_OVERFLOW, FSDA_E_WORKSPACE,
 * FSDA_E_CSR, FSDA_E_LABELS, FSDA_E_HIP.
 */
int fsda_build_operator(const fsda_problem *pb, int max_shifts, int max_chunk, void *workspace,
                        size_t ws_bytes, void *stream, fsda_op **out);

/*
 * Right-hand side of Alg. 7, step 4, into b[d] (device, FP64).
 *  r == NULL: the canonical b = (X - 1 mu_l^T)^T y_c = X^T y_c, y_c the labels
 *             minus their labeled mean (0 on unlabeled samples);
 *  r != NULL: r[d] (device) is the start vector of Alg. 7, step 2, and
 *             b = (X - 1 mu_l^T)^T [W 0; 0 0] X r with W_ij = 1/N_c on the
 *             labeled class blocks (Sec. 2.1).  For two classes this equals
 *             ((m+ - m-)/2) X^T y_c, m_c the class-c mean of X r.
 */
int fsda_rhs(fsda_op *op, const double *r, double *b, void *stream);

/*
 * q = A(sigma) p for one vector (the operator product inside each Krylov
 * step, Sec. 3.2.3): p[d], q[d] device FP64, sigma >= 0 host.  The centring is
 * applied once, as a rank-one correction in sample space.
 */
int fsda_apply(fsda_op *op, double sigma, const double *p, double *q, void *stream);

/*
 * Multi-shift solve (Alg. 3): one conjugate-gradient recurrence on
 * A(min beta), every other shift carried by the collinear-residual
 * coefficients zeta relative to it (Sec. 3.2.2).  The per-shift direction
 * coefficient is formed with the freshly computed CG coefficient b_{i+1}, the
 * reading under which the shifted residuals stay collinear.
 *  b[d]        device FP64 right-hand side, or NULL for the canonical one.
 *  betas[nshift] host, each > 0, 1 <= nshift <= max_shifts of the handle.
 *  rtol        > 0: shift s stops updating once |zeta_s| ||r|| <= rtol ||b||.
 *  maxit       >= 1 iterations of the shared recurrence.
 *  chunk       1..max_chunk: iterations between folds of the per-shift state
 *              and between host checks for termination (0 = default 128,
 *              capped at max_chunk).  The recurrence, the iteration counts and
 *              the stopping points do not depend on chunk; W does only through
 *              the order of its rounding (a chunk's per-shift updates are
 *              applied as one linear combination of its residuals).
 *  W[nshift][d] device FP64 output, w_s for beta_s.
 *  iters[nshift] host int output: iterations after which shift s stopped
 *              (FSDA_MIXED: plus the iterations of its correction solves).
 *  relres[nshift] host FP64 output: true residual ||b - A(beta_s) w_s|| / ||b||
 *              recomputed in FP64 from w_s after the solve.
 * Returns FSDA_OK, FSDA_NOT_CONVERGED (some shift hit maxit; its w_s is the
 * last iterate), FSDA_E_BREAKDOWN, or an argument error.  Blocks until done.
 *
 * FSDA_MIXED: the shared recurrence runs with FP32 vectors (FP64 dot products
 * and scalars) to max(rtol, 1e-5), where FP32 rounding stalls it; then one
 * step of FP64 iterative refinement: R_s = b - A(beta_s) w_s in FP64, the
 * corrections A(beta_s) delta_s = R_s of every shift not yet within rtol solved
 * at once by batched FP32 CG (one column per shift; the residuals of different
 * shifts are not collinear, so they cannot share one shifted basis) to
 * 0.5 rtol ||b|| (at most 1e-6 below ||R_s||), and w_s += delta_s in FP64.  The
 * status is FSDA_OK when every reported relres[s] <= rtol, else
 * FSDA_NOT_CONVERGED.
 */
int fsda_multishift_solve(fsda_op *op, const double *b, const double *betas, int nshift, double rtol, int maxit,
                          int chunk, double *W, int *iters, double *relres, void *stream);

/*
 * Breakdown of the last completed fsda_multishift_solve on this handle, per
 * shift (host outputs of nshift entries; nshift must be that solve's):
 * main_iters[s] the iterations after which shift s stopped in the shared
 * recurrence, refine_iters[s] the iterations of its correction solve
 * (FSDA_MIXED; 0 otherwise), steps[s] the refinement steps it took (0 or 1).
 * iters[s] of the solve is main_iters[s] + refine_iters[s].  Host only.
 */
int fsda_solve_report(const fsda_op *op, int nshift, int *main_iters, int *refine_iters, int *steps);

/*
 * Spectral analysis for SDA (Alg. sasda): the ratings of the samples present
 * in X come straight from the sample-space system
 *     (Cl^T M + beta I_N) z = g,   Cl = I_N - 1 1_l^T / l,
 * M = (1-alpha) P_l + alpha L, solved for every beta by the same shared-basis
 * recurrence (Alg. 3) over vectors of length n; the rating is s = z.  Cl^T M
 * is the symmetric centred weight M' (the centring lands on the labeled rows
 * only), so no X product is involved.  With alpha = 0 the unlabeled ratings
 * are 0, so alpha > 0 is the useful range (alpha = 0 is not rejected).
 * Always FP64, whatever the handle's precision.
 *
 * fsda_sa_rhs: g[n] (device) = y_c (r == NULL, canonical) or the printed
 *   right-hand side [W 0; 0 0](r - 1 <1_l, r>/l) for the start vector r[n]
 *   (device), which for two classes equals ((m+ - m-)/2) y_c, m_c the mean of
 *   r over the labeled rows of class c.
 * fsda_sa_solve: g[n] device (NULL = canonical y_c); betas, nshift, rtol,
 *   maxit, chunk as in fsda_multishift_solve; Z[nshift][n] device FP64 output
 *   (the ratings); iters, relres host as in fsda_multishift_solve (relres the
 *   true FP64 residual ||g - (M' + beta_s I) z_s|| / ||g||).  Blocks until done.
 */
int fsda_sa_rhs(fsda_op *op, const double *r, double *g, void *stream);
int fsda_sa_solve(fsda_op *op, const double *g, const double *betas, int nshift, double rtol, int maxit, int chunk,
                  double *Z, int *iters, double *relres, void *stream);

/*
 * Regression phase of the spectral-regression variants (Alg. optimizedSR,
 * step 5; Alg. SR, step 6): (X^T X + beta I_D) w = X^T z for every beta, z[n]
 * a sample-space vector (device, e.g. the ratings of fsda_sa_solve).  No
 * graph, no centring, no labels (the handle's are not used).  shared_basis
 * != 0: one recurrence for all shifts (Alg. 3); 0: an independent CG per
 * shift (the baseline of Table tab:shifted), each stopping at its own rtol.
 * betas, nshift, rtol, maxit, chunk, W[nshift][d], iters, relres as in
 * fsda_multishift_solve (relres relative to ||X^T z||).  Always FP64.
 * Blocks until done.
 */
int fsda_regression_solve(fsda_op *op, const double *z, const double *betas, int nshift, double rtol, int maxit,
                          int chunk, int shared_basis, double *W, int *iters, double *relres, void *stream);

/*
 * Many targets at once (the shared-basis solve of Sec. 3.2.2 applied to
 * several binary labelings of the same samples, e.g. one per assay): target c
 * has its own labeled set, hence its own centred operator
 *     A_c(beta) = X^T [ (1-alpha)(P_lc - 1_lc 1_lc^T / l_c) + alpha L ] X + beta I
 * and right-hand side b_c = X^T y_c (the canonical one of fsda_rhs for that
 * labeled set), and is solved for every beta of one grid by its own shifted
 * CG (Alg. 3, seeded at min beta), in FP64.  X, S and alpha are the
 * handle's; its own labeled set is not used.  Targets go in tiles of up to
 * 16 (fsda_set_batch_tile, fsda_batch_autotune), one tile after the other; the
 * sparse products of the targets of a tile share one pass over the indices.
 * The rows of X^T of >= 512 nonzeros are summed in pieces and the shorter
 * ones one group of lanes each (FSDA_BXT_MED sets the boundary); the longest
 * rows (>= 16 nonzeros per slice on average) are summed from slices of the
 * sample-space vector staged in LDS (FSDA_BXT_LDS_SEG sets that threshold, 0
 * turns it off); when the sample-space vector over a tile's targets outgrows
 * an XCD's share of L2 (n x tile x 8 bytes > 2 MiB), the other pieces of rows
 * of >= 2 chunks are summed in XCD slices (each XCD gathers from one eighth of
 * the samples; FSDA_BXT_SLICES set to 0 or 8 overrides this).  The X^T
 * product also does the residual update (r -= a q and its partial sums; in the
 * column solves the iterate update as well) unless FSDA_BXT_FUSE=0.  These
 * environment variables apply here and in the column solves, and must be the
 * same for the workspace-size call.  With FSDA_PROGRESS=<seconds> the host
 * loops of every solve print their iteration count to stderr at most that
 * often (read when a handle is built).
 *  ntarget       1..FSDA_MAX_TARGETS.
 *  lab_idx[], lab_y[] (device) the labeled sets of all targets, concatenated;
 *                target c owns entries lab_off[c] .. lab_off[c+1]-1 (same
 *                rules as the handle's labeled set: in range, no repeats,
 *                labels +1/-1, both classes present).
 *  lab_off[ntarget+1] host offsets, lab_off[0] = 0.
 *  betas, nshift, rtol, maxit, chunk: as in fsda_multishift_solve (1 <= nshift
 *                <= FSDA_MAX_SHIFTS; the handle's max_shifts does not apply;
 *                0 <= chunk <= FSDA_MAX_BATCH_CHUNK, 0 = default 96; as there,
 *                chunk changes W only through the order of its rounding).
 *  workspace     device, 256-byte aligned, ws_bytes >= fsda_batch_workspace_size()
 *                for the same ntarget, nshift and chunk; scratch for this call only.
 *  W[ntarget][nshift][d] device FP64 output.
 *  iters[ntarget * nshift], relres[ntarget * nshift] host outputs, per (target,
 *                shift), relres the true FP64 residual relative to ||b_c||.
 * Errors as fsda_multishift_solve; FSDA_E_LABELS names the offending target.
 * Blocks until done.
 */
int fsda_batch_workspace_size(const fsda_op *op, int ntarget, int nshift, int chunk, size_t *bytes);
int fsda_multishift_solve_batch(fsda_op *op, int ntarget, const int32_t *lab_idx, const int8_t *lab_y,
                                const int64_t *lab_off, const double *betas, int nshift, double rtol, int maxit,
                                int chunk, void *workspace, size_t ws_bytes, double *W, int *iters, double *relres,
                                void *stream);

/*
 * Launch shape of fsda_multishift_solve_batch (not part of the method): the
 * targets per tile T (a tile of T targets shares one pass over the indices per
 * sparse product; its vectors over samples are interleaved, T values per row)
 * and the groups of T lanes that share one row of the row products (the X and
 * graph products and the short rows of X^T), so a wave holds 64 / (T groups)
 * rows.
 *  fsda_set_batch_tile: tile 4, 8 or 16, or 0 for the default (16).  Takes
 *                effect at the next fsda_batch_workspace_size and batch solve
 *                (the workspace size depends on it).
 *  fsda_set_batch_groups: groups 1, 2 or 4, or 0 for the default (1).
 *  Errors: FSDA_E_ARG, FSDA_E_RANGE.  The getters write the shape in use to
 *  *tile, *groups (host).
 */
int fsda_set_batch_tile(fsda_op *op, int tile);
int fsda_get_batch_tile(const fsda_op *op, int *tile);
int fsda_set_batch_groups(fsda_op *op, int groups);
int fsda_get_batch_groups(const fsda_op *op, int *groups);

/*
 * Autotuner of the launch shape: for each tile T in {4, 8, 16} not larger than
 * the tile that min(ntarget, 16) targets need, and each group count in {1, 2,
 * 4}, solves the first min(T, ntarget) targets (arguments as in
 * fsda_multishift_solve_batch) once to warm up (graph capture), then for
 * trial_iters and 2 trial_iters iterations (rtol 1e-300, so nothing stops
 * early), and takes the time difference of the last two over their iteration
 * difference: setup and the final residual checks cancel.  rates[9] (host)
 * receive the shifted target-iterations per second of (tile, groups) = (4, 1),
 * (4, 2), (4, 4), (8, 1), ..., (16, 4) (0 where not tried); the fastest shape
 * is kept in the handle (as by fsda_set_batch_tile and fsda_set_batch_groups)
 * and written to *tile, *groups.  Blocks until done.
 *  trial_iters   1..4096 (32 to 64 suffice on the benchmark workloads).
 *  workspace, ws_bytes  as for fsda_multishift_solve_batch with the default
 *                tile (16) and the same ntarget, nshift and chunk 0.
 *  W             device FP64, room for min(ntarget, 16) x nshift x d; its
 *                contents afterwards are the unconverged trial iterates.
 * Errors as fsda_multishift_solve_batch (the shape in use before the call is
 * kept then), and FSDA_E_RANGE for trial_iters.
 */
int fsda_batch_autotune(fsda_op *op, int ntarget, const int32_t *lab_idx, const int8_t *lab_y,
                        const int64_t *lab_off, const double *betas, int nshift, int trial_iters, void *workspace,
                        size_t ws_bytes, double *W, void *stream, int *tile, int *groups, double *rates);

/*
 * Independent systems with different right-hand sides, solved together:
 *     A(sigma_c) x_c = b_c,  c < ncol,  A(sigma) = X^T M' X + sigma I
 * (the handle's operator; e.g. the adjoint systems of the hypergradient, whose
 * right-hand sides differ per shift, so one shifted basis cannot serve them).
 * Batched CG in FP64, one column per system, the sparse products of all
 * columns sharing one pass over the indices.
 *  B[ncol][d]   device, right-hand sides in the caller's feature order.
 *  sigmas[ncol] host, each > 0.   ncol 1..FSDA_MAX_COLUMNS.
 *  rtol, maxit  column c stops when ||r_c|| <= rtol ||b_c||; at most maxit iterations.
 *  workspace    device, 256-byte aligned, >= fsda_columns_workspace_size(); scratch.
 *  X[ncol][d]   device FP64 output.   iters, relres[ncol] host (true FP64 residual).
 * Blocks until done.
 */
int fsda_columns_workspace_size(const fsda_op *op, int ncol, size_t *bytes);
int fsda_solve_columns(fsda_op *op, const double *B, const double *sigmas, int ncol, double rtol, int maxit,
                       void *workspace, size_t ws_bytes, double *X, int *iters, double *relres, void *stream);

/*
 * fsda_solve_columns without a workspace argument, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * hosts that forbid allocation): the same solve and results, with its scratch
 * in a static device array of FSDA_STATIC_SCRATCH_BYTES that the library holds
 * on every GPU it is loaded on until the process ends.  The call allocates
 * nothing (no device allocation, no graph instantiation: its kernels are
 * launched directly).  Arguments and outputs as fsda_solve_columns.
 * Scratch needed: fsda_columns_workspace_size(); a solve that needs more is
 * rejected with FSDA_E_WORKSPACE before any HIP call.  All calls on one GPU
 * share that GPU's scratch: calls that overlap in time on one GPU (two
 * streams, two threads, two handles) race and give wrong results.  Blocks
 * until done.
 */
#define FSDA_STATIC_SCRATCH_BYTES (64u << 20)
int fsda_solve_columns_static(fsda_op *op, const double *B, const double *sigmas, int ncol, double rtol, int maxit,
                              double *X, int *iters, double *relres, void *stream);

/*
 * Hold-out loss of the ratings (Alg. 7, return value) for selecting beta and
 * alpha:  H_s = 1/2 ||X_ho w_s - y_ho||^2 / n_ho for every row w_s of W.
 *  W[nshift][d]  device, caller's feature order (e.g. from fsda_multishift_solve).
 *  ho_idx[n_ho]  device int32 held-out rows (distinct, in range); ho_y[n_ho] device FP64 targets.
 *  loss[nshift]  host output.
 *  G[nshift][d]  device output or NULL: the gradient of H_s in w_s,
 *                X_ho^T (X_ho w_s - y_ho) / n_ho, the right-hand side of the
 *                adjoint system A(beta_s) lambda_s = G_s (fsda_solve_columns).
 * FSDA_E_ARG for a held-out index out of range or repeated.  Blocks until done.
 */
int fsda_holdout(fsda_op *op, const double *W, int nshift, const int32_t *ho_idx, const double *ho_y, int64_t n_ho,
                 double *loss, double *G, void *stream);

/*
 * Hypergradient of the hold-out loss from the solutions W and the adjoint
 * solutions Lambda (A symmetric: A(beta_s) lambda_s = G_s):
 *     dH_s/d log beta_s = -beta_s <lambda_s, w_s>
 *     dH_s/d alpha      = -<X lambda_s, [L - (P_l - 1_l 1_l^T / l)] X w_s>
 * (A is affine in alpha with that slope; b does not depend on either).
 *  W, Lambda[nshift][d] device, caller's order; betas[nshift] host.
 *  dlogbeta[nshift], dalpha[nshift] host outputs.  Blocks until done.
 */
int fsda_hypergradient(fsda_op *op, const double *W, const double *Lambda, const double *betas, int nshift,
                       double *dlogbeta, double *dalpha, void *stream);

/*
 * Many targets (as in fsda_multishift_solve_batch): the hold-out loss, the
 * adjoint systems and the hypergradient of every (target, shift), for
 * selecting beta and alpha per target over held-out labeled data (the ratings
 * of Alg. 7 judged on labels the solve did not see).  Arrays over (target,
 * shift) are ordered c * nshift + s; W, G, Lambda are [ntarget][nshift][d] in
 * the caller's feature order.
 *
 * fsda_holdout_batch: loss[c * nshift + s] (host) = 1/2 ||X_ho,c w_cs -
 *   y_ho,c||^2 / n_ho,c with target c's held-out rows ho_idx[ho_off[c] ..
 *   ho_off[c+1]) (device int32, distinct within a target, in range) and targets
 *   ho_y (device FP64, same positions); ho_off[ntarget+1] host, ho_off[0] = 0,
 *   at least one held-out row per target.  G (device, or NULL) receives
 *   X_ho,c^T (X_ho,c w_cs - y_ho,c) / n_ho,c, the right-hand sides of the
 *   adjoint systems.  FSDA_E_ARG names the target of a bad held-out index.
 *
 * fsda_solve_columns_batch: solves A_c(beta_s) lambda_cs = B_cs for every
 *   (target, shift), A_c the operator of target c's labeled set (lab_idx,
 *   lab_y, lab_off as in fsda_multishift_solve_batch: the training part of
 *   each target's labels) with the handle's X, S and alpha.  The right-hand
 *   sides differ per (target, shift), so no shared basis: batched CG in FP64,
 *   columns in tiles of 16 (each tile's products one pass over the indices),
 *   taken shift by shift (the columns of one tile share a shift, so they need
 *   similar iteration counts), tiles one after the other.  B, X [ntarget][nshift][d] device; betas
 *   [nshift] host, each > 0; rtol, maxit per column as in fsda_solve_columns;
 *   workspace device, 256-byte aligned, >= fsda_columns_batch_workspace_size()
 *   (one tile; scratch); iters, relres [ntarget * nshift] host (relres the
 *   true FP64 residual relative to ||B_cs||).  Status: the worst over the
 *   columns (FSDA_NOT_CONVERGED if any column reached maxit).  Blocks until
 *   done.
 *
 * fsda_hypergradient_batch: from W and Lambda (A_c symmetric, so Lambda solves
 *   the transposed system too), dlogbeta[c * nshift + s] = -beta_s <lambda_cs,
 *   w_cs> and dalpha[c * nshift + s] = -<X lambda_cs, [L - (P_lc - 1_lc 1_lc^T
 *   / l_c)] X w_cs> (host outputs), with target c's training labeled set.
 * 1 <= ntarget <= FSDA_MAX_TARGETS, 1 <= nshift <= FSDA_MAX_SHIFTS.
 */
int fsda_holdout_batch(fsda_op *op, int ntarget, const double *W, int nshift, const int32_t *ho_idx,
                       const double *ho_y, const int64_t *ho_off, double *loss, double *G, void *stream);
int fsda_columns_batch_workspace_size(const fsda_op *op, int ntarget, int nshift, size_t *bytes);
int fsda_solve_columns_batch(fsda_op *op, int ntarget, const int32_t *lab_idx, const int8_t *lab_y,
                             const int64_t *lab_off, const double *betas, int nshift, const double *B, double rtol,
                             int maxit, void *workspace, size_t ws_bytes, double *X, int *iters, double *relres,
                             void *stream);
int fsda_hypergradient_batch(fsda_op *op, int ntarget, const int32_t *lab_idx, const int8_t *lab_y,
                             const int64_t *lab_off, const double *W, const double *Lambda, const double *betas,
                             int nshift, double *dlogbeta, double *dalpha, void *stream);

/*
 * Ratings s = X w for each shift (Alg. 7, return value; uncentred):
 * W[nshift][d] device FP64 in, S[nshift][n] device FP64 out.
 */
int fsda_project(fsda_op *op, const double *W, int nshift, double *S, void *stream);

/*
 * Per-kernel timing for measurement: enable >= 1 makes the handle record a
 * pair of HIP events around every enable-th launch (the first, then every
 * enable-th after it; 1 = every launch) of the kernel class `kernel` on the
 * launch stream; enable = 0 switches timing off, a negative value is
 * FSDA_E_RANGE.  Classes: 0 = X product, 1 = graph/centring product, 2 = X^T
 * product (fused with the residual update of every short row of X^T in the
 * feature-space solves; with LDS slices it also finishes the split rows),
 * 3 = the LDS-slice part of the X^T product (k_xt_lds), 4 = residual update (sample-space solves), 5 =
 * direction update (feature space with X^T unsliced: also the residual update
 * of the rows of X^T longer than one chunk; with XCD slices those rows are
 * finished between classes 2 and 5, in class 13), 6 = shift-state fold; the batched FP32 correction solves of FSDA_MIXED: 7 = X
 * product, 8 = graph/centring product, 9 = X^T product, 10 = residual and
 * correction update (no launches where the X^T product does it), 11 =
 * direction update; fsda_multishift_solve_batch: 7-9
 * its products, 10 = residual update (no launches where the X^T product does
 * it), 11 = direction update, 12 = shift-state fold; 13 = the assembly of the X^T rows cut into XCD slices (their parts
 * summed, then the residual update of those rows).  While timing is on, solves launch kernels
 * directly instead of replaying a graph.  Launches made after the recurrence
 * stopped (which return at once) are not counted.  fsda_kernel_time() returns
 * (host) the summed milliseconds and count of the timed launches since the
 * last reset and resets them.
 */
int fsda_time_kernel(fsda_op *op, int kernel, int enable);
int fsda_kernel_time(fsda_op *op, double *ms, int64_t *launches);

/*
 * Measurement aid (no part of the method): partials[b] = the sum of src[idx[k]]
 * over the k that block b of `grid` blocks takes (grid-stride, 256 threads per
 * block, 8 independent gathers in flight per thread), enqueued on `stream`.
 * It measures the rate of random 8-byte gathers, the resource the sparse
 * products of the solve are bound by.  src (device FP64), idx[nidx] (device
 * int32, every entry in [0, length of src): not checked), partials[grid]
 * (device FP64, written).  nidx >= 0, 1 <= grid <= 65536, else FSDA_E_RANGE;
 * NULL partials (or NULL src/idx with nidx > 0) is FSDA_E_ARG.
 */
int fsda_gather_sum(const double *src, const int *idx, int64_t nidx, double *partials, int grid, void *stream);

/* Frees the host handle (and its events); the caller frees the workspace. */
void fsda_destroy_operator(fsda_op *op);

/* Message for the last negative status returned on this thread. */
const char *fsda_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FSDA_H */
