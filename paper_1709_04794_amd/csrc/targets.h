// Many binary targets over one sample set: T labelings of the same X and S
// (each with its own labeled set, hence its own centring and right-hand side)
// solved together over one shift grid.  Every target runs its own shifted CG
// (Alg. 3, seeded at the smallest shift); the sparse products of all T targets
// share one pass over the indices (the batched products of batched.h, in FP64).
//
// Layout: the vectors the products gather from (the direction P, and t, u in
// sample space) are interleaved, element (row j, target c) at j * T + c.  The
// vectors that are only streamed (the residual ring R, the product Q, the
// right-hand sides B, and the per-shift state W_s, P_s) are column-major,
// element (c, j) at c * ld + j (W and P_s at (c * S + s) * ld + j), so the
// shift fold sees one target per block and reads its coefficients as
// wave-uniform values.
#pragma once

#include "batched.h"

namespace fsda {

constexpr int TS_MAX = 64;  // shifts per target
constexpr int SBS = 1024;   // threads of the one-block scalar steps (they sum thousands of partials per column)

struct TState {
  int iter, stop, status, maxit;
  int ncol, nshift, chunk, fold_start;
  int zero;                        // always 0: the stop flag of launches outside the recurrence
  int pad_[3];
  double* W;                       // the caller's [ncol][nshift][d] iterates (read by the fold, so
                                   // that one captured chunk serves every tile of a call)
  double rr[BT_MAX];               // <r_c, r_c>
  double a_cur[BT_MAX], a_prev[BT_MAX], b_cur[BT_MAX];
  double tol[BT_MAX];              // rtol ||b_c||
  double bnorm[BT_MAX];
  double sigma[BT_MAX];            // seed shift (the smallest beta), the same for every target
  double cm[BT_MAX];               // labeled mean of t_c
  int col_active[BT_MAX];
  double rel[TS_MAX];              // beta_s - sigma0
  // per (target, shift), index c * TS_MAX + s
  double zp[BT_MAX * TS_MAX], z[BT_MAX * TS_MAX], zn[BT_MAX * TS_MAX], as[BT_MAX * TS_MAX];
  double res2[BT_MAX * TS_MAX];    // ||b_c - A_c(beta_s) w_cs||^2 after the solve
  int active[BT_MAX * TS_MAX];
  int conv[BT_MAX * TS_MAX];
};

// Column-major streaming kernels run on a (gx, T) grid: block (x, c) covers
// the rows j = x * BS + tid, x * BS + tid + gx * BS, ... of target c, and
// writes one partial per block into part[x * T + c].
template <int T>
__device__ __forceinline__ void write_partial_col(double* part, double acc) {
  const double t = block_sum_all(acc);
  if (threadIdx.x == 0) part[(size_t)blockIdx.x * T + blockIdx.y] = t;
}

// ---------------------------------------------------------------------------
// set-up
// ---------------------------------------------------------------------------

// Pass 1 over the labeled entries [k0, k1) of target c: range, repeats (cnt is
// an n x T counter, zero on entry), label values, class counts into
// flags[c * 4 + {0: positives, 1: negatives, 2: error bits}].
template <int T>
__global__ void tk_label_check(const int* idx, const int8_t* y, long long k0, long long k1, int c, long long n,
                               int* cnt, int* flags) {
  FSDA_GRID_LOOP(kk, k1 - k0) {
    const long long k = k0 + kk;
    const int i = idx[k];
    if (i < 0 || i >= n) {
      atomicOr(&flags[c * 4 + 2], 1);
      continue;
    }
    if (atomicAdd(&cnt[(size_t)i * T + c], 1) != 0) atomicOr(&flags[c * 4 + 2], 2);
    const int yy = y[k];
    if (yy == 1)
      atomicAdd(&flags[c * 4 + 0], 1);
    else if (yy == -1)
      atomicAdd(&flags[c * 4 + 1], 1);
    else
      atomicOr(&flags[c * 4 + 2], 4);
  }
}

// Pass 2: labw[i * T + c] = 1/l_c, ycen[i * T + c] = y_i - mean_c(y) on the
// labeled rows of target c (the arrays are zero elsewhere).
template <int T>
__global__ void tk_label_vectors(const int* idx, const int8_t* y, long long k0, long long k1, int c, double inv_l,
                                 double ybar, double* labw, double* ycen) {
  FSDA_GRID_LOOP(kk, k1 - k0) {
    const long long k = k0 + kk;
    const int i = idx[k];
    labw[(size_t)i * T + c] = inv_l;
    ycen[(size_t)i * T + c] = (y[k] > 0 ? 1.0 : -1.0) - ybar;
  }
}

// ---------------------------------------------------------------------------
// recurrence
// ---------------------------------------------------------------------------

// ring slot 0 = B_c, P = B (interleaved), P_s = B_c, W_s = 0 (targets c < ncol
// only; W is the caller's [ncol][nshift][d]); partials of <b_c, b_c>.
template <int T>
__global__ __launch_bounds__(BS) void ts_init(const double* __restrict__ B, long long ld, double* ring, double* P,
                                              double* Ps, double* W, long long d, int ncol, int nshift,
                                              double* part) {
  const int c = blockIdx.y;
  double acc = 0.0;
  for (long long j = (long long)blockIdx.x * BS + threadIdx.x; j < d; j += (long long)gridDim.x * BS) {
    const double x = B[(size_t)c * ld + j];
    ring[(size_t)c * ld + j] = x;
    P[(size_t)j * T + c] = x;
    if (c < ncol)
      for (int s = 0; s < nshift; s++) {
        Ps[((size_t)c * nshift + s) * ld + j] = x;
        W[((size_t)c * nshift + s) * d + j] = 0.0;
      }
    acc += x * x;
  }
  write_partial_col<T>(part, acc);
}

// rr_c, ||b_c||, tolerances, the zeta windows; a target with a zero right-hand
// side (or a padding column) never starts.  One block.
template <int T>
__global__ __launch_bounds__(BS) void ts_init_done(TState* st, const double* part, int np) {
  __shared__ double rr[T];
  __shared__ int any;
  col_sums<T>(part, np, rr);
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  const int S = st->nshift;
  for (int e = threadIdx.x; e < T * S; e += BS) {
    const int c = e / S, s = e % S, k = c * TS_MAX + s;
    const int on = c < st->ncol && rr[c] > 0.0;
    st->zp[k] = 1.0;
    st->z[k] = 1.0;
    st->active[k] = on;
    st->conv[k] = 0;
  }
  if (threadIdx.x < T) {
    const int c = threadIdx.x;
    const int on = c < st->ncol && rr[c] > 0.0;
    st->rr[c] = rr[c];
    st->bnorm[c] = sqrt(rr[c]);
    st->tol[c] = st->tol[c] * st->bnorm[c];  // held rtol
    st->a_prev[c] = 1.0;
    st->b_cur[c] = 0.0;
    st->a_cur[c] = 0.0;
    st->col_active[c] = on;
    if (on) atomicOr(&any, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0 && !any) st->stop = 1;
}

// a_c = rr_c / (<t,u>_c + sigma0 <p,p>_c) (<p_0, p_0> = <b, b> = rr_c in the
// first iteration); the zeta step of every active (target, shift):
// zeta_{i+1} and a_s = a zeta_{i+1} / zeta_i.  One block.
template <int T>
__global__ __launch_bounds__(SBS) void ts_step_a(TState* st, const double* tu_part, int ntu, const double* pp_part,
                                                int npp) {
  if (st->stop) return;
  __shared__ double tu[T], pp[T], av[T];
  __shared__ int bad;
  col_sums<T, SBS>(tu_part, ntu, tu);
  col_sums<T, SBS>(pp_part, npp, pp);
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  if (threadIdx.x < T) {
    const int c = threadIdx.x;
    double a = 0.0;
    if (st->col_active[c]) {
      const double ppc = st->iter == 0 ? st->rr[c] : pp[c];
      const double pq = tu[c] + st->sigma[c] * ppc;
      a = st->rr[c] / pq;
      if (!(pq > 0.0) || !isfinite(a)) {
        atomicOr(&bad, 1);
        a = 0.0;
      }
    }
    av[c] = a;
  }
  __syncthreads();
  if (bad) {
    if (threadIdx.x == 0) {
      st->status = FSDA_E_BREAKDOWN;
      st->stop = 1;
    }
    return;
  }
  const int S = st->nshift;
  for (int e = threadIdx.x; e < T * S; e += SBS) {
    const int c = e / S, s = e % S, k = c * TS_MAX + s;
    if (!st->active[k]) continue;
    const double a = av[c], ap = st->a_prev[c], b = st->b_cur[c];
    const double zp = st->zp[k], z = st->z[k];
    const double den = a * b * (zp - z) + zp * ap * (1.0 + st->rel[s] * a);
    const double zn = zp * z * ap / den;
    st->zn[k] = zn;
    st->as[k] = a * zn / z;
  }
  if (threadIdx.x < T) st->a_cur[threadIdx.x] = av[threadIdx.x];
}

// r_{i+1} = r_i - a_c q (ring slots i % m and (i + 1) % m, column-major);
// partials of <r_{i+1}, r_{i+1}>.  Grid (gx, T).
template <int T>
__global__ __launch_bounds__(BS) void ts_resid(const TState* st, const double* __restrict__ Q, double* ring,
                                               long long ld, long long d, double* part) {
  if (st->stop) return;
  const int c = blockIdx.y;
  const int i = st->iter, m = st->chunk;
  const double a = st->a_cur[c];
  const double* r = ring + ((size_t)(i % m) * T + c) * ld;
  double* rn = ring + ((size_t)((i + 1) % m) * T + c) * ld;
  const double* q = Q + (size_t)c * ld;
  double acc = 0.0;
  for (long long j = (long long)blockIdx.x * BS + threadIdx.x; j < d; j += (long long)gridDim.x * BS) {
    const double x = r[j] - a * q[j];
    rn[j] = x;
    acc += x * x;
  }
  write_partial_col<T>(part, acc);
}

// b_c = rr'/rr; per (target, shift): the fold coefficients (a_s, zeta_{i+1},
// b_s = b (zeta_{i+1}/zeta_i)^2, 1), or the identity (0, 0, 1, 0) once frozen,
// into hist[((i % m) * T + c) * S + s]; the stop test |zeta_{i+1}| ||r_{i+1}||
// <= rtol ||b_c||; target and global stop; iteration count.  One block.
template <int T>
__global__ __launch_bounds__(SBS) void ts_step_b(TState* st, const double* rr_part, int nrr, double* hist) {
  if (st->stop) return;
  __shared__ double rrn[T], bv[T];
  __shared__ int still[T];
  __shared__ int any;
  col_sums<T, SBS>(rr_part, nrr, rrn);
  if (threadIdx.x < T) {
    const int c = threadIdx.x;
    bv[c] = st->col_active[c] ? rrn[c] / st->rr[c] : 0.0;
    still[c] = 0;
  }
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  const int i = st->iter, S = st->nshift, slot = i % st->chunk;
  for (int e = threadIdx.x; e < T * S; e += SBS) {
    const int c = e / S, s = e % S, k = c * TS_MAX + s;
    double* h = hist + (((size_t)slot * T + c) * S + s) * 4;
    if (st->active[k]) {
      const double zn = st->zn[k], z = st->z[k];
      const double ratio = zn / z;
      h[0] = st->as[k];
      h[1] = zn;
      h[2] = bv[c] * ratio * ratio;
      h[3] = 1.0;
      st->zp[k] = z;
      st->z[k] = zn;
      st->conv[k] = i + 1;
      if (fabs(zn) * sqrt(rrn[c]) <= st->tol[c])
        st->active[k] = 0;
      else
        atomicOr(&still[c], 1);
    } else {
      h[0] = 0.0;
      h[1] = 0.0;
      h[2] = 1.0;
      h[3] = 0.0;
    }
  }
  __syncthreads();
  if (threadIdx.x < T) {
    const int c = threadIdx.x;
    if (st->col_active[c]) {
      st->a_prev[c] = st->a_cur[c];
      st->b_cur[c] = bv[c];
      st->rr[c] = rrn[c];
      st->col_active[c] = still[c];
      if (still[c]) atomicOr(&any, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st->iter = i + 1;
    if (!any) {
      st->stop = 1;
    } else if (i + 1 >= st->maxit) {
      st->stop = 1;
      st->status = FSDA_NOT_CONVERGED;
    }
  }
}

// P = r_{i+1} + b_c P (interleaved; the ring is column-major) for the targets
// still active; partials of <p, p> per target.
template <int T>
// r_{i+1} is column-major in the ring and P interleaved: a block takes RT rows
// at a time, reads their T columns of r whole (RT consecutive values per
// column) into LDS, then updates P row by row from there.
__global__ __launch_bounds__(BS) void ts_pupdate(const TState* st, const double* __restrict__ ring, long long ld,
                                                 double* P, long long d, double* part) {
  if (st->stop) return;
  constexpr int G = BS / T;
  constexpr int RT = 4 * G;  // rows per pass: T RT = 4 BS values of r
  __shared__ double tile[T][RT + 1];
  const int c = threadIdx.x % T, g = threadIdx.x / T;
  const double b = st->b_cur[c];
  const bool on = st->col_active[c] != 0;
  const double* r0 = ring + (size_t)((st->iter) % st->chunk) * T * ld;  // iter was advanced by ts_step_b
  double acc = 0.0;
  for (long long j0 = (long long)blockIdx.x * RT; j0 < d; j0 += (long long)gridDim.x * RT) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int e = threadIdx.x + k * BS, cc = e / RT, jj = e % RT;
      tile[cc][jj] = j0 + jj < d ? r0[(size_t)cc * ld + j0 + jj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 4; m++) {
      const int jj = g + m * G;
      const long long j = j0 + jj;
      if (j < d) {
        const size_t e = (size_t)j * T + c;
        double p = P[e];
        if (on) {
          p = tile[c][jj] + b * p;
          P[e] = p;
        }
        acc += p * p;
      }
    }
    __syncthreads();
  }
  write_partials_cols<T>(part, acc);
}

// Fold of iterations [fold_start, iter) into the state of every (target,
// shift), as in the single-target solve: the chunk's steps
//   W_s += a_k P_s ;  P_s = zeta_k r_k + b_k P_s
// unrolled into W_s <- W_s + A_s P_s + sum_k H_k,s r_k, P_s <- B_s P_s + sum_k G_k,s r_k.
// ts_fold_coef: one block per target (blockIdx.y), one thread per shift, the
// coefficients backwards over the chunk into coef[c] = {H [cnt][S], G [cnt][S],
// A [S], B [S], on [S]}; ts_fold_apply: grid (gx, ncol), the target's buffered
// residuals streamed once per group of TFG shifts.
constexpr int TFG = 16;  // shifts per pass over a target's buffered residuals
__host__ __device__ inline size_t ts_coef_stride(int chunk, int nshift) {
  return (size_t)(2 * chunk + 3) * nshift;  // doubles per target
}

__global__ __launch_bounds__(BS) void ts_fold_coef(const TState* st, const double* __restrict__ hist, int T,
                                                   double* __restrict__ coef, int nshift) {
  const int k0 = st->fold_start, cnt = st->iter - k0, m = st->chunk;
  const int c = blockIdx.y, s = threadIdx.x;
  if (cnt <= 0 || s >= nshift || c >= st->ncol) return;
  double* H = coef + (size_t)c * ts_coef_stride(m, nshift);
  double* G = H + (size_t)m * nshift;
  double* AB = G + (size_t)m * nshift;  // A [S], B [S], on [S]
  constexpr int KB = 16;
  double gp = 0.0, e = 1.0;
  for (int kb = cnt - 1; kb >= 0; kb -= KB) {
    double a[KB], z[KB], b[KB];
#pragma unroll
    for (int u = 0; u < KB; u++) {
      const int k = kb - u >= 0 ? kb - u : 0;
      const double* h = hist + ((((size_t)((k0 + k) % m)) * T + c) * nshift + s) * 4;
      a[u] = h[0];
      z[u] = h[1];
      b[u] = h[2];
    }
#pragma unroll
    for (int u = 0; u < KB; u++) {
      const int k = kb - u;
      if (k >= 0) {
        H[(size_t)k * nshift + s] = z[u] * gp;
        G[(size_t)k * nshift + s] = z[u] * e;
        gp = a[u] + b[u] * gp;
        e = b[u] * e;
      }
    }
  }
  AB[s] = gp;
  AB[nshift + s] = e;
  AB[2 * nshift + s] = hist[((((size_t)(k0 % m)) * T + c) * nshift + s) * 4 + 3] != 0.0 ? 1.0 : 0.0;
}

__global__ __launch_bounds__(BS) void ts_fold_apply(const TState* st, const double* __restrict__ coef, int T,
                                                    const double* ring, long long ld, double* Ps, long long d,
                                                    int nshift) {
  const int k0 = st->fold_start, cnt = st->iter - k0, m = st->chunk;
  const int c = blockIdx.y;
  if (cnt <= 0 || c >= st->ncol) return;
  double* W = st->W;
  const double* H = coef + (size_t)c * ts_coef_stride(m, nshift);
  const double* G = H + (size_t)m * nshift;
  const double* AB = G + (size_t)m * nshift;
  const int first = (k0 + 1) % m;
  constexpr int KU = 8;  // buffered residuals in flight
  // the group's coefficients staged once per block and read as broadcasts (as
  // scalar operands the KU x TFG x 2 coefficients of an unrolled step outgrow
  // the SGPRs); the launch's LDS holds m rows of TFG
  extern __shared__ double tfold_lds[];
  double* lh = tfold_lds;
  double* lg = tfold_lds + (size_t)m * TFG;
  for (int s0 = 0; s0 < nshift; s0 += TFG) {
    __syncthreads();
    for (int e = threadIdx.x; e < cnt * TFG; e += BS) {
      const int k = e / TFG, s = s0 + e % TFG;
      lh[e] = s < nshift ? H[(size_t)k * nshift + s] : 0.0;
      lg[e] = s < nshift ? G[(size_t)k * nshift + s] : 0.0;
    }
    __syncthreads();
    for (long long j = (long long)blockIdx.x * BS + threadIdx.x; j < d; j += (long long)gridDim.x * BS) {
      double ah[TFG], ag[TFG];
#pragma unroll
      for (int g = 0; g < TFG; g++) ah[g] = ag[g] = 0.0;
      for (int k = 0; k < cnt; k += KU) {
        double rv[KU];
#pragma unroll
        for (int u = 0; u < KU; u++) {  // slot (k0 + k + u + 1) mod m: the chunk wraps the ring at most once
          const int sl = first + k + u;
          rv[u] = k + u < cnt ? ring[((size_t)(sl < m ? sl : sl - m) * T + c) * ld + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < KU; u++) {
          if (k + u < cnt) {
            const double* hk = lh + (size_t)(k + u) * TFG;
            const double* gk = lg + (size_t)(k + u) * TFG;
#pragma unroll
            for (int g = 0; g < TFG; g++) {
              ah[g] += hk[g] * rv[u];
              ag[g] += gk[g] * rv[u];
            }
          }
        }
      }
#pragma unroll
      for (int g = 0; g < TFG; g++) {
        const int s = s0 + g;
        if (s < nshift && AB[2 * nshift + s] != 0.0) {
          const size_t e = (size_t)c * nshift + s;
          const double pv = Ps[e * ld + j];
          W[e * d + j] += AB[s] * pv + ah[g];
          Ps[e * ld + j] = AB[nshift + s] * pv + ag[g];
        }
      }
    }
  }
}

// LDS of ts_fold_apply for a fold interval of m iterations (rows rounded up to
// a multiple of 4 for ts_fold_apply_mfma).
inline size_t ts_fold_lds_bytes(int m) { return 2 * sizeof(double) * (size_t)((m + 3) / 4 * 4) * TFG; }

// The same fold on the matrix cores.  For a target c and a group of 16 shifts
// the chunk's sums over the buffered residuals are a small dense product,
//   [sum_k H_k,s r_k(j)]_{s,j} = H^T (16 x cnt) R (cnt x columns),
// and likewise with G: each wave takes 16 columns j at a time and accumulates
// them with the FP64 16x16x4 instruction, 4 buffered residuals per step.  Lane
// layout of that instruction (checked on gfx950): lane l supplies A[l % 16][l /
// 16] and B[l / 16][l % 16], and holds D[l / 16 + 4 v][l % 16] in element v.
// Here A[i][kk] = H[k][s0 + i] (from LDS, zero beyond cnt and nshift), B[kk][jj]
// = r_k(j0 + jj) (zero beyond cnt and d), k = 4 kb + kk; lane l then finishes
// shifts s0 + l / 16 + 4 v of column j0 + l % 16.  Every instruction runs with
// all 64 lanes (the loops are uniform over the wave; only loads and stores are
// predicated).
typedef double tf_d4 __attribute__((ext_vector_type(4)));
constexpr int TFK = 4;  // steps of 4 buffered residuals whose loads are in flight together
__global__ __launch_bounds__(BS) void ts_fold_apply_mfma(const TState* st, const double* __restrict__ coef, int T,
                                                         const double* ring, long long ld, double* Ps, long long d,
                                                         int nshift) {
  const int k0 = st->fold_start, cnt = st->iter - k0, m = st->chunk;
  const int c = blockIdx.y;
  if (cnt <= 0 || c >= st->ncol) return;
  double* W = st->W;
  const double* H = coef + (size_t)c * ts_coef_stride(m, nshift);
  const double* G = H + (size_t)m * nshift;
  const double* AB = G + (size_t)m * nshift;
  const int first = (k0 + 1) % m;
  const int nkb = (cnt + 3) / 4;
  extern __shared__ double tfold_lds[];
  double* lh = tfold_lds;  // [4 nkb][16]
  double* lg = tfold_lds + (size_t)(m + 3) / 4 * 4 * TFG;
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  constexpr int WPB = BS / 64;  // waves per block
  const long long jstep = (long long)gridDim.x * WPB * 16;
  for (int s0 = 0; s0 < nshift; s0 += TFG) {
    __syncthreads();
    for (int e = threadIdx.x; e < nkb * 4 * TFG; e += BS) {
      const int k = e / TFG, s = s0 + e % TFG;
      const bool ok = k < cnt && s < nshift;
      lh[e] = ok ? H[(size_t)k * nshift + s] : 0.0;
      lg[e] = ok ? G[(size_t)k * nshift + s] : 0.0;
    }
    __syncthreads();
    for (long long j0 = ((long long)blockIdx.x * WPB + (threadIdx.x >> 6)) * 16; j0 < d; j0 += jstep) {
      const long long j = j0 + li;
      const bool jin = j < d;
      tf_d4 dh = {0.0, 0.0, 0.0, 0.0}, dg = {0.0, 0.0, 0.0, 0.0};
      for (int kb0 = 0; kb0 < nkb; kb0 += TFK) {
        double rv[TFK];
#pragma unroll
        for (int u = 0; u < TFK; u++) {  // slot (k0 + k + 1) mod m: the chunk wraps the ring at most once
          const int k = (kb0 + u) * 4 + lk;
          const int sl = first + k;
          rv[u] = k < cnt && jin ? ring[((size_t)(sl < m ? sl : sl - m) * T + c) * ld + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < TFK; u++) {
          if (kb0 + u < nkb) {  // uniform over the wave
            const int e = ((kb0 + u) * 4 + lk) * TFG + li;
            dh = __builtin_amdgcn_mfma_f64_16x16x4f64(lh[e], rv[u], dh, 0, 0, 0);
            dg = __builtin_amdgcn_mfma_f64_16x16x4f64(lg[e], rv[u], dg, 0, 0, 0);
          }
        }
      }
      if (jin) {
#pragma unroll
        for (int v = 0; v < 4; v++) {
          const int s = s0 + lk + 4 * v;
          if (s < nshift && AB[2 * nshift + s] != 0.0) {
            const size_t e = (size_t)c * nshift + s;
            const double pv = Ps[e * ld + j];
            W[e * d + j] += AB[s] * pv + dh[v];
            Ps[e * ld + j] = AB[nshift + s] * pv + dg[v];
          }
        }
      }
    }
  }
}

__global__ void ts_fold_done(TState* st) { st->fold_start = st->iter; }

// ---------------------------------------------------------------------------
// after the solve
// ---------------------------------------------------------------------------

// P[j * T + c] = W[(c * nshift + s) * d + j] for c < ncol, 0 for the padding columns.
template <int T>
__global__ __launch_bounds__(BS) void ts_pack(const double* __restrict__ W, int s, int nshift, int ncol, double* P,
                                              long long d) {
  constexpr int G = BS / T;
  const int c = threadIdx.x % T, g = threadIdx.x / T;
  for (long long j = (long long)blockIdx.x * G + g; j < d; j += (long long)gridDim.x * G)
    P[(size_t)j * T + c] = c < ncol ? W[((size_t)c * nshift + s) * d + j] : 0.0;
}

// partials of ||B_c - Q_c - beta w_cs||^2 (Q = X^T M' X w_cs, column-major).  Grid (gx, ncol).
template <int T>
__global__ __launch_bounds__(BS) void ts_resnorm(const double* __restrict__ B, const double* __restrict__ Q,
                                                 long long ld, const double* __restrict__ W, int s, int nshift,
                                                 double beta, long long d, double* part) {
  const int c = blockIdx.y;
  const double* w = W + ((size_t)c * nshift + s) * d;
  double acc = 0.0;
  for (long long j = (long long)blockIdx.x * BS + threadIdx.x; j < d; j += (long long)gridDim.x * BS) {
    const double r = B[(size_t)c * ld + j] - (Q[(size_t)c * ld + j] + beta * w[j]);
    acc += r * r;
  }
  write_partial_col<T>(part, acc);
}

// res2[c * TS_MAX + s] = sum of the partials of target c.  One block.
template <int T>
__global__ __launch_bounds__(BS) void ts_res_done(TState* st, const double* part, int np, int s, int ncol) {
  __shared__ double v[T];
  col_sums<T>(part, np, v);
  if (threadIdx.x < ncol) st->res2[threadIdx.x * TS_MAX + s] = v[threadIdx.x];
}

// out[(row) * d + jj] = W[row * d + old2new[jj]] for rows [r0, r1) of W ([ncol * nshift][d]).
__global__ void ts_unpermute(const double* __restrict__ W, const int* __restrict__ old2new, double* out, long long r0,
                             long long r1, long long d) {
  FSDA_GRID_LOOP(e, (r1 - r0) * d) {
    const long long row = r0 + e / d, jj = e % d;
    out[e] = W[row * d + old2new[jj]];
  }
}

}  // namespace fsda
