// Device code of the multi-shift SDA solver (gfx950, wave64).
//
// Everything on this path is bound by memory bandwidth or latency: the sparse
// products are gather-sums over int32 column indices of binary matrices (no
// multiplies), the rest are streaming vector updates and FP64 dot products.
// No kernel here is a dense contraction, so none uses the matrix cores.
//
// Reductions never synchronise blocks inside a kernel.  A producing kernel
// writes one partial per block; every block of the consuming kernel sums the
// partials itself in the same fixed order (so all blocks hold the same bits),
// and the last block to finish (taken with a relaxed ticket: it reads nothing
// the other blocks wrote in that kernel) updates the solver state, which the
// following kernels read.  No device-scope fence, hence no L2 write-back, sits
// on the critical path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fsda.h"

namespace fsda {

constexpr int BS = 256;       // threads per block (4 waves of 64)
constexpr int TILE = 2048;    // nonzeros per row-complete tile
constexpr int CAP = 4096;     // values a tile stages (split tiles hold exactly CAP)
constexpr int IPT = CAP / BS; // nonzeros per thread in a tile
constexpr int ROWCAP = 2048;  // row pointers a tile stages
constexpr int MAXS = 64;      // shifts per handle
constexpr int MAXCHUNK = 64;  // iterations per shift-state fold
constexpr int NPART = 4096;   // partials per reduction site
constexpr int MAXBIN = 8;     // row-length bins of a row product
constexpr int UNR = 4;        // independent loads per thread in streaming loops

enum Site { SITE_X = 0, SITE_XT = 1, SITE_R = 2, SITE_INIT = 3, NSITE = 4 };

// Solver state, resident in device memory.
struct State {
  unsigned int ticket[8];  // last-block counters
  int iter;                // iterations of the shared recurrence completed
  int stop;                // every shift stopped, maxit, or breakdown
  int status;              // 0 ok, 1 maxit reached, -5 breakdown
  int fold_start;          // first iteration not yet folded into W, P
  int nshift, maxit, chunk, pad_;
  double rr;               // <r_i, r_i>
  double tol;              // rtol * ||b||
  double bnorm;
  double a_cur, a_prev;    // CG step lengths a_i, a_{i-1} (a_i = -gamma_i of Alg. 3)
  double b_cur;            // CG direction coefficient b_i (alpha_i of Alg. 3)
  double sig[MAXS];        // beta_s - sigma0
  double zp[MAXS], z[MAXS], zn[MAXS];  // zeta_{i-1}, zeta_i, zeta_{i+1}
  double as[MAXS], bs[MAXS];           // per-shift step and direction coefficients
  double res2[MAXS];       // ||b - A(beta_s) w_s||^2 after the solve
  int active[MAXS];
  int conv[MAXS];          // iteration at which shift s stopped
};

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sum in a fixed order; every thread gets the result.
__device__ __forceinline__ double block_sum_all(double v) {
  __shared__ double sh[BS / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < BS / 64; i++) t += sh[i];
  return t;
}

// Sum of the n partials a previous kernel wrote (fixed order; every thread
// of every block computes the same bits).
__device__ __forceinline__ double sum_partials(const double* part, int n) {
  double v = 0.0;
  constexpr int U = 8;
  for (int i0 = threadIdx.x; i0 < n; i0 += BS * U) {
    double x[U];
#pragma unroll
    for (int u = 0; u < U; u++) x[u] = (i0 + u * BS < n) ? part[i0 + u * BS] : 0.0;
#pragma unroll
    for (int u = 0; u < U; u++) v += x[u];
  }
  return block_sum_all(v);
}

__device__ __forceinline__ void write_partial(double* part, int slot, double acc) {
  const double t = block_sum_all(acc);
  if (threadIdx.x == 0) part[slot] = t;
}

// True in every thread of the last block to reach it.
__device__ __forceinline__ bool last_block(unsigned int* ticket) {
  __shared__ int amlast;
  __syncthreads();
  if (threadIdx.x == 0) amlast = atomicAdd(ticket, 1u) == gridDim.x - 1;
  __syncthreads();
  return amlast != 0;
}

// ---------------------------------------------------------------------------
// scalar recurrences: thread s of the last block handles shift s
// ---------------------------------------------------------------------------

// a_i known: collinearity factor zeta_{i+1} of Alg. 3 and step a_s = a_i zeta_{i+1}/zeta_i.
__device__ void step_scalars(State* st, double a) {
  const double ap = st->a_prev, b = st->b_cur;
  const int s = threadIdx.x;
  if (s < st->nshift && st->active[s]) {
    const double zp = st->zp[s], z = st->z[s];
    const double den = a * b * (zp - z) + zp * ap * (1.0 + st->sig[s] * a);
    const double zn = zp * z * ap / den;
    st->zn[s] = zn;
    st->as[s] = a * zn / z;
  }
  if (threadIdx.x == 0) st->a_cur = a;
}

// r_{i+1} known: b_{i+1} = rrn/rr, per-shift direction coefficient
// b_s = b_{i+1} (zeta_{i+1}/zeta_i)^2 (Alg. 3 with the fresh coefficient), the
// coefficients recorded for the fold, the per-shift stop test
// |zeta_{i+1}| ||r_{i+1}|| <= rtol ||b||, and the shift of the zeta window.
__device__ void resid_scalars(State* st, double rrn, double b, double* hist) {
  const int i = st->iter;
  const double rn = sqrt(rrn);
  const int slot = i % st->chunk;
  const int s = threadIdx.x;
  int still = 0;
  if (s < st->nshift) {
    double* h = hist + ((size_t)slot * MAXS + s) * 4;
    if (st->active[s]) {
      const double zn = st->zn[s], z = st->z[s];
      const double ratio = zn / z;
      const double bs = b * ratio * ratio;
      st->bs[s] = bs;
      h[0] = st->as[s];
      h[1] = zn;
      h[2] = bs;
      h[3] = 1.0;
      st->zp[s] = z;
      st->z[s] = zn;
      if (fabs(zn) * rn <= st->tol) {
        st->active[s] = 0;
        st->conv[s] = i + 1;
      } else {
        still = 1;
        if (i + 1 >= st->maxit) st->conv[s] = i + 1;
      }
    } else {
      h[3] = 0.0;
    }
  }
  const int any = __syncthreads_or(still);
  if (threadIdx.x == 0) {
    st->a_prev = st->a_cur;
    st->b_cur = b;
    st->rr = rrn;
    st->iter = i + 1;
    if (!any) {
      st->stop = 1;
    } else if (i + 1 >= st->maxit) {
      st->stop = 1;
      st->status = FSDA_NOT_CONVERGED;
    }
  }
}

// ---------------------------------------------------------------------------
// row epilogues of the sparse products
// ---------------------------------------------------------------------------

// t = X p; with W, reduction sum_r w_r t_r (w = 1/l on labeled rows gives their mean).
template <bool W>
struct EpiX {
  double* t;
  const double* w;
  static constexpr bool kReduce = W;
  __device__ void prepare(const State*) {}
  __device__ double row(int r, double v) const {
    t[r] = v;
    return W ? w[r] * v : 0.0;
  }
};

// u = M' t = (1-alpha)[r labeled](t_r - c) + alpha (d_r t_r - (S t)_r): the
// weight of Eq. SDAeig with the centring of Sec. 3.2.3 applied once, in sample
// space.  c (the labeled mean of t) is the sum of the X product's partials.
template <bool LAB>
struct EpiLap {
  const double* t;
  const double* labw;
  const int* srowptr;
  double* u;
  double alpha;
  const double* cpart;
  int ncpart;
  double c;
  static constexpr bool kReduce = false;
  __device__ void prepare(const State*) { c = LAB ? sum_partials(cpart, ncpart) : 0.0; }
  __device__ double row(int r, double v) const {
    const double tr = t[r];
    const double deg = (double)(srowptr[r + 1] - srowptr[r]);
    double x = alpha * (deg * tr - v);
    if (LAB && labw[r] != 0.0) x += (1.0 - alpha) * (tr - c);
    u[r] = x;
    return 0.0;
  }
};

// q = X^T u + sigma p; reduction <p, q>.
template <bool RED>
struct EpiXT {
  double* q;
  const double* p;
  double sigma;
  static constexpr bool kReduce = RED;
  __device__ void prepare(const State*) {}
  __device__ double row(int r, double v) const {
    const double pr = p ? p[r] : 0.0;
    const double qq = v + sigma * pr;
    q[r] = qq;
    return pr * qq;
  }
};

// True residual of one shift: R = b - (X^T u + beta w); reduction ||R||^2.
struct EpiRes {
  const double* b;
  const double* w;
  double beta;
  static constexpr bool kReduce = true;
  __device__ void prepare(const State*) {}
  __device__ double row(int r, double v) const {
    const double R = b[r] - (v + beta * w[r]);
    return R * R;
  }
};

// ---------------------------------------------------------------------------
// sparse products, lanes per row
// ---------------------------------------------------------------------------
//
// Rows are grouped in bins of similar length (for X^T the features are
// relabeled by decreasing frequency, so the bins are contiguous row ranges).
// In a bin, `lpr` lanes share a row and take UNR nonzeros each per pass: all
// index loads, then all gathers, are in flight together; the lanes then add up
// with shuffles.  lpr == 0 marks rows known to be empty.

struct Rows {
  const int* rowptr;
  const int* col;
  int nb;
  int row0[MAXBIN + 1];
  int lpr[MAXBIN];
  int item0[MAXBIN + 1];  // work items before bin b; an item is BS/lpr rows (BS when lpr == 0)
};

template <class Epi>
__global__ __launch_bounds__(BS) void k_rows(Rows R, const double* __restrict__ src, Epi epi, State* st,
                                             double* part, int slot0, int solve) {
  if (solve && st->stop) return;
  epi.prepare(st);
  const int tid = threadIdx.x;
  double acc = 0.0;
  const int nitems = R.item0[R.nb];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    int b = 0;
    while (it >= R.item0[b + 1]) b++;
    const int lpr = R.lpr[b];
    if (lpr == 0) {
      const int r = R.row0[b] + (it - R.item0[b]) * BS + tid;
      if (r < R.row0[b + 1]) acc += epi.row(r, 0.0);
      continue;
    }
    const int r = R.row0[b] + (it - R.item0[b]) * (BS / lpr) + tid / lpr;
    const int lane = tid & (lpr - 1);
    const bool live = r < R.row0[b + 1];
    double v = 0.0;
    if (live) {
      const int beg = R.rowptr[r], end = R.rowptr[r + 1];
      for (int k0 = beg + lane; k0 < end; k0 += lpr * UNR) {
        int idx[UNR];
        double g[UNR];
#pragma unroll
        for (int u = 0; u < UNR; u++) {
          const int k = k0 + u * lpr;
          idx[u] = k < end ? R.col[k] : -1;
        }
#pragma unroll
        for (int u = 0; u < UNR; u++) g[u] = idx[u] >= 0 ? src[idx[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < UNR; u++) v += g[u];
      }
    }
    for (int o = lpr >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (live && lane == 0) acc += epi.row(r, v);
  }
  if (Epi::kReduce) write_partial(part, slot0 + blockIdx.x, acc);
}

// ---------------------------------------------------------------------------
// sparse products over nonzero tiles (long rows)
// ---------------------------------------------------------------------------
//
// The nonzeros of rows [0, nrows) are cut into tiles of `tile` entries.  Tile
// b owns the rows whose first nonzero lies in it.
//  - row-complete mode: the block stages all of its own rows, even past the
//    tile end (rows are at most CAP - TILE long), so each row finishes in one
//    block;
//  - split mode: the block stages exactly its tile; the partial sum of the row
//    entering the tile goes to head[b], that of its last row leaving the tile
//    to tail[b], and k_fixup finishes those rows from the heads of the tiles
//    they cover.
// In a tile, each thread takes IPT consecutive nonzeros, finds the row of the
// first one by binary search over the tile's row pointers (staged in LDS) and
// walks its values, splitting them at row ends; a block-wide segmented scan
// hands every thread the partial sum of the row its values continue, and the
// thread holding a row's last value finishes it.  Work per thread is the same
// whatever the row lengths.

struct Tiles {
  const int* rowptr;
  const int* col;
  int nrows;
  long long nnz;
  const int* tile_row;  // [ntiles+1]
  const int* cross;     // [ntiles] row leaving tile b, or -1 (split mode)
  int ntiles;
  int split;
  int tile;
  double* head;
  double* tail;
};

__device__ __forceinline__ void seg_combine(int fa, double va, int& fb, double& vb) {
  if (!fb) vb += va;
  fb |= fa;
}

// Exclusive segmented scan of (flag, value) over the block in thread order.
__device__ __forceinline__ double block_seg_exscan(int f, double v) {
  __shared__ double wv[BS / 64];
  __shared__ int wf[BS / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int fi = f;
  double vi = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double vo = __shfl_up(vi, o, 64);
    const int fo = __shfl_up(fi, o, 64);
    if (lane >= o) seg_combine(fo, vo, fi, vi);
  }
  double ve = __shfl_up(vi, 1, 64);
  int fe = __shfl_up(fi, 1, 64);
  if (lane == 0) {
    ve = 0.0;
    fe = 0;
  }
  __syncthreads();
  if (lane == 63) {
    wf[w] = fi;
    wv[w] = vi;
  }
  __syncthreads();
  int fp = 0;
  double vp = 0.0;
  for (int k = 0; k < w; k++) {
    int fk = wf[k];
    double vk = wv[k];
    seg_combine(fp, vp, fk, vk);
    fp = fk;
    vp = vk;
  }
  seg_combine(fp, vp, fe, ve);
  return ve;
}

__device__ __forceinline__ int padi(int j) { return j + (j >> 4); }

template <class Epi>
__global__ __launch_bounds__(BS) void k_tiles(Tiles tl, const double* __restrict__ src, Epi epi, State* st,
                                              double* part, int slot0, int solve) {
  if (solve && st->stop) return;
  __shared__ double vals[CAP + CAP / 16];
  __shared__ int rps[ROWCAP + 1];
  epi.prepare(st);
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int b = blockIdx.x; b < tl.ntiles; b += gridDim.x) {
    const long long lo = (long long)b * tl.tile;
    const long long hi = min(lo + (long long)tl.tile, tl.nnz);
    const int r0 = tl.tile_row[b], r1 = tl.tile_row[b + 1];
    const long long rs0 = tl.rowptr[r0];
    long long beg, end;
    if (tl.split) {
      beg = lo;
      end = hi;
    } else {
      beg = rs0;
      end = tl.rowptr[r1];
    }
    const int cnt = (int)(end - beg);
    const bool head = tl.split && (beg < rs0);
    const int first = head ? r0 - 1 : r0;
    const int nr = r1 - first;  // rows touching the tile, empty owned rows included
    const bool fast = nr + 1 <= ROWCAP;
    {
      int idx[IPT];
      double gv[IPT];
#pragma unroll
      for (int it = 0; it < IPT; it++) {
        const int k = it * BS + tid;
        idx[it] = (k < cnt) ? tl.col[beg + k] : -1;
      }
#pragma unroll
      for (int it = 0; it < IPT; it++) gv[it] = (idx[it] >= 0) ? src[idx[it]] : 0.0;
#pragma unroll
      for (int it = 0; it < IPT; it++) {
        const int k = it * BS + tid;
        if (k < cnt) vals[padi(k)] = gv[it];
      }
    }
    if (fast)
      for (int i = tid; i <= nr; i += BS) rps[i] = tl.rowptr[first + i];
    __syncthreads();
    const int crossing = tl.split ? tl.cross[b] : -1;
    if (fast) {
      const int ia = tid * IPT;
      const int ib = min(ia + IPT, cnt);
      const bool has = ia < cnt;
      const int ga = (int)beg + ia;
      double x[IPT];
#pragma unroll
      for (int i = 0; i < IPT; i++) x[i] = (ia + i < cnt) ? vals[padi(ia + i)] : 0.0;
      int s0 = 0;
      if (has) {  // largest s with rps[s] <= ga
        int l = 0, h = nr - 1;
        while (l < h) {
          const int m = (l + h + 1) >> 1;
          if (rps[m] <= ga) l = m; else h = m - 1;
        }
        s0 = l;
      }
      const bool starts_here = has && rps[s0] == ga;
      int flag = starts_here ? 1 : 0;
      double run = 0.0;
      {
        int s = s0;
#pragma unroll
        for (int i = 0; i < IPT; i++) {
          if (ia + i < ib) {
            const int g = ga + i;
            if (g >= rps[s + 1]) {
              flag = 1;
              do s++; while (rps[s + 1] <= g);
              run = 0.0;
            }
            run += x[i];
          }
        }
      }
      const double carry = block_seg_exscan(has ? flag : 0, has ? run : 0.0);
      if (has) {
        int s = s0;
        double v = starts_here ? 0.0 : carry;
        auto finish = [&](int sr, double tot) {
          const int r = first + sr;
          if (head && sr == 0)
            tl.head[b] = tot;
          else if (r == crossing)
            tl.tail[b] = tot;
          else
            acc += epi.row(r, tot);
        };
#pragma unroll
        for (int i = 0; i < IPT; i++) {
          if (ia + i < ib) {
            const int g = ga + i;
            if (g >= rps[s + 1]) {
              finish(s, v);
              do s++; while (rps[s + 1] <= g);
              v = 0.0;
            }
            v += x[i];
          }
        }
        if (rps[s + 1] <= ga + (ib - ia) || ib == cnt) finish(s, v);
      }
      for (int i = (head ? 1 : 0) + tid; i < nr; i += BS)
        if (rps[i] == rps[i + 1]) acc += epi.row(first + i, 0.0);
    } else {
      for (int i = tid; i < nr; i += BS) {
        const int r = first + i;
        const long long sb = max((long long)tl.rowptr[r], beg);
        const long long se = min((long long)tl.rowptr[r + 1], end);
        double v0 = 0.0, v1 = 0.0;
        long long k = sb;
        for (; k + 1 < se; k += 2) {
          v0 += vals[padi((int)(k - beg))];
          v1 += vals[padi((int)(k + 1 - beg))];
        }
        if (k < se) v0 += vals[padi((int)(k - beg))];
        const double v = v0 + v1;
        if (head && i == 0)
          tl.head[b] = v;
        else if (r == crossing)
          tl.tail[b] = v;
        else
          acc += epi.row(r, v);
      }
    }
    if (tl.split && !head && tid == 0) tl.head[b] = 0.0;
    __syncthreads();
  }
  if (Epi::kReduce) write_partial(part, slot0 + blockIdx.x, acc);
}

template <class Epi>
__global__ __launch_bounds__(BS) void k_fixup(Tiles tl, Epi epi, State* st, double* part, int slot0, int solve) {
  if (solve && st->stop) return;
  epi.prepare(st);
  double acc = 0.0;
  for (int b = blockIdx.x * BS + threadIdx.x; b < tl.ntiles; b += gridDim.x * BS) {
    const int r = tl.cross[b];
    if (r < 0) continue;
    const long long e = tl.rowptr[r + 1];
    double v = tl.tail[b];
    for (long long bb = b + 1; bb * tl.tile < e; bb++) v += tl.head[bb];
    acc += epi.row(r, v);
  }
  if (Epi::kReduce) write_partial(part, slot0 + blockIdx.x, acc);
}

// ---------------------------------------------------------------------------
// streaming kernels of the recurrence
// ---------------------------------------------------------------------------

// r_0 = b (ring slot 0), p_0 = b, P_s = b, W_s = 0; partials of <b, b>.
__global__ __launch_bounds__(BS) void k_init(const double* __restrict__ b, double* ring, double* p, double* P,
                                             long long ldp, double* W, long long d, int nshift, double* part) {
  double acc = 0.0;
  for (long long j = (long long)blockIdx.x * BS + threadIdx.x; j < d; j += (long long)gridDim.x * BS) {
    const double x = b[j];
    ring[j] = x;
    p[j] = x;
    for (int s = 0; s < nshift; s++) {
      P[s * ldp + j] = x;
      W[s * d + j] = 0.0;
    }
    acc += x * x;
  }
  write_partial(part, blockIdx.x, acc);
}

// rr = <b,b>, tol = rtol ||b||; a zero right-hand side stops at once.  One block.
__global__ __launch_bounds__(BS) void k_init_done(State* st, const double* part, int np) {
  const double all = sum_partials(part, np);
  if (threadIdx.x == 0) {
    st->rr = all;
    st->bnorm = sqrt(all);
    st->tol = st->tol * st->bnorm;  // st->tol held rtol
    if (!(all > 0.0)) {
      st->stop = 1;
      for (int s = 0; s < st->nshift; s++) {
        st->active[s] = 0;
        st->conv[s] = 0;
      }
    }
  }
}

// K4: a_i = <r,r>/<p,q> from the X^T product's partials; r_{i+1} = r_i - a_i q
// into the next ring slot; partials of <r_{i+1}, r_{i+1}>.  The last block
// advances zeta (or flags a breakdown).
__global__ __launch_bounds__(BS) void k_resid(State* st, const double* __restrict__ q, double* ring, long long ldd,
                                              long long d, const double* pq_part, int npq, double* part) {
  if (st->stop) return;
  const double pq = sum_partials(pq_part, npq);
  const int i = st->iter, m = st->chunk;
  const double a = st->rr / pq;
  const bool ok = (pq > 0.0) && isfinite(a);
  double acc = 0.0;
  if (ok) {
    const double* r = ring + (long long)(i % m) * ldd;
    double* rn = ring + (long long)((i + 1) % m) * ldd;
    const long long step = (long long)gridDim.x * BS * UNR;
    for (long long j0 = (long long)blockIdx.x * BS * UNR + threadIdx.x; j0 < d; j0 += step) {
      double rv[UNR], qv[UNR];
#pragma unroll
      for (int u = 0; u < UNR; u++) {
        const long long j = j0 + (long long)u * BS;
        rv[u] = j < d ? r[j] : 0.0;
        qv[u] = j < d ? q[j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UNR; u++) {
        const long long j = j0 + (long long)u * BS;
        const double x = rv[u] - a * qv[u];
        if (j < d) rn[j] = x;
        acc += x * x;
      }
    }
  }
  write_partial(part, blockIdx.x, acc);
  if (last_block(&st->ticket[SITE_R])) {
    if (ok) {
      step_scalars(st, a);
    } else if (threadIdx.x == 0) {
      st->status = FSDA_E_BREAKDOWN;
      st->stop = 1;
    }
    if (threadIdx.x == 0) st->ticket[SITE_R] = 0;
  }
}

// K5: b_{i+1} = <r_{i+1},r_{i+1}>/<r_i,r_i>; p_{i+1} = r_{i+1} + b_{i+1} p_i.  The
// last block runs the per-shift scalar updates and the stop test.
__global__ __launch_bounds__(BS) void k_pupdate(State* st, const double* ring, double* p, long long ldd, long long d,
                                                const double* rr_part, int nrr, double* hist) {
  if (st->stop) return;
  const double rrn = sum_partials(rr_part, nrr);
  const int i = st->iter;
  const double b = rrn / st->rr;
  const double* r = ring + (long long)((i + 1) % st->chunk) * ldd;
  const long long step = (long long)gridDim.x * BS * UNR;
  for (long long j0 = (long long)blockIdx.x * BS * UNR + threadIdx.x; j0 < d; j0 += step) {
    double rv[UNR], pv[UNR];
#pragma unroll
    for (int u = 0; u < UNR; u++) {
      const long long j = j0 + (long long)u * BS;
      rv[u] = j < d ? r[j] : 0.0;
      pv[u] = j < d ? p[j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UNR; u++) {
      const long long j = j0 + (long long)u * BS;
      if (j < d) p[j] = rv[u] + b * pv[u];
    }
  }
  if (last_block(&st->ticket[SITE_INIT])) {
    resid_scalars(st, rrn, b, hist);
    if (threadIdx.x == 0) st->ticket[SITE_INIT] = 0;
  }
}

// Fold of iterations [fold_start, iter): per element, keep the buffered
// residuals in registers and replay, shift by shift, the recurrences
//   W_s += a_s P_s ;  P_s = zeta_{k+1,s} r_{k+1} + b_s P_s
// exactly as a per-iteration pass would, in the same order.  Shifts go in
// groups of SG so that their W and P loads are in flight together.
constexpr int SG = 4;
template <int M>
__global__ __launch_bounds__(BS) void k_fold(const State* st, const double* __restrict__ hist, const double* ring,
                                             long long ldd, double* W, long long d, double* P, long long ldp,
                                             int nshift) {
  // (a_s, zeta, b_s) and the active flag of every (iteration, shift) of the
  // chunk, in dynamic LDS sized by the host for chunk * nshift entries
  extern __shared__ double dyn[];
  const int k0 = st->fold_start, k1 = st->iter, m = st->chunk;
  const int cnt = k1 - k0;
  if (cnt <= 0) return;
  double* co = dyn;
  int* act = reinterpret_cast<int*>(dyn + 3 * m * nshift);
  for (int e = threadIdx.x; e < cnt * nshift; e += BS) {
    const int k = e / nshift, s = e % nshift;
    const double* h = hist + ((size_t)((k0 + k) % m) * MAXS + s) * 4;
    co[e * 3 + 0] = h[0];
    co[e * 3 + 1] = h[1];
    co[e * 3 + 2] = h[2];
    act[e] = h[3] != 0.0;
  }
  __syncthreads();
  for (long long j = (long long)blockIdx.x * BS + threadIdx.x; j < d; j += (long long)gridDim.x * BS) {
    double rv[M];
#pragma unroll
    for (int k = 0; k < M; k++)
      if (k < cnt) rv[k] = ring[(long long)((k0 + k + 1) % m) * ldd + j];
    for (int s0 = 0; s0 < nshift; s0 += SG) {
      double w[SG], pp[SG];
#pragma unroll
      for (int g = 0; g < SG; g++) {
        const int s = s0 + g;
        const bool on = s < nshift && act[s];  // inactive at the chunk start -> stays inactive
        w[g] = on ? W[s * d + j] : 0.0;
        pp[g] = on ? P[s * ldp + j] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < M; k++) {
        if (k < cnt) {
#pragma unroll
          for (int g = 0; g < SG; g++) {
            const int s = s0 + g;
            if (s < nshift && act[k * nshift + s]) {
              const double* c = co + (k * nshift + s) * 3;
              w[g] += c[0] * pp[g];
              pp[g] = c[1] * rv[k] + c[2] * pp[g];
            }
          }
        }
      }
#pragma unroll
      for (int g = 0; g < SG; g++) {
        const int s = s0 + g;
        if (s < nshift && act[s]) {
          W[s * d + j] = w[g];
          P[s * ldp + j] = pp[g];
        }
      }
    }
  }
}

__global__ void k_fold_done(State* st) { st->fold_start = st->iter; }

// out = sum of np partials (one block).
__global__ __launch_bounds__(BS) void k_sum_to(const double* part, int np, double* out) {
  const double all = sum_partials(part, np);
  if (threadIdx.x == 0) *out = all;
}

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------

#define FSDA_GRID_LOOP(j, n) \
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < (n); j += (long long)gridDim.x * blockDim.x)

__global__ void k_fill_d(double* x, long long n, double v) { FSDA_GRID_LOOP(j, n) x[j] = v; }
__global__ void k_fill_i(int* x, long long n, int v) { FSDA_GRID_LOOP(j, n) x[j] = v; }
__global__ void k_iota(int* x, long long n) { FSDA_GRID_LOOP(j, n) x[j] = (int)j; }
// dst[j] = src[map[j]]
__global__ void k_gather_d(const double* __restrict__ src, const int* __restrict__ map, double* dst, long long n) {
  FSDA_GRID_LOOP(j, n) dst[j] = src[map[j]];
}
// dst[j] = f * sum(partials) * src[map[j]]
__global__ __launch_bounds__(BS) void k_gather_scaled_d(const double* __restrict__ src, const int* __restrict__ map,
                                                        double* dst, long long n, const double* part, int np,
                                                        double f) {
  const double c = f * sum_partials(part, np);
  FSDA_GRID_LOOP(j, n) dst[j] = c * src[map[j]];
}
__global__ void k_gather_i(const int* __restrict__ src, const int* __restrict__ map, int* dst, long long n) {
  FSDA_GRID_LOOP(j, n) dst[j] = map[src[j]];
}
// inverse permutation: inv[perm[j]] = j
__global__ void k_invert(const int* perm, int* inv, long long n) { FSDA_GRID_LOOP(j, n) inv[perm[j]] = (int)j; }

// flag bits: 1 rowptr not monotone / out of [0, nnz], 16 rowptr[0] != 0 or rowptr[n] != nnz.
__global__ void k_check_rowptr(const int* rowptr, long long nrows, long long nnz, int* flag) {
  FSDA_GRID_LOOP(r, nrows) {
    const long long a = rowptr[r], b = rowptr[r + 1];
    if (a < 0 || a > b || b > nnz) atomicOr(flag, 1);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    if (rowptr[0] != 0 || (long long)rowptr[nrows] != nnz) atomicOr(flag, 16);
}

// flag bits: 2 column out of range, 4 not strictly increasing, 8 self loop.
__global__ void k_check_cols(const int* rowptr, const int* col, long long nrows, long long ncols, int noself,
                             int* flag) {
  FSDA_GRID_LOOP(r, nrows) {
    const int a = rowptr[r], b = rowptr[r + 1];
    int prev = -1;
    int f = 0;
    for (int k = a; k < b; k++) {
      const int c = col[k];
      if (c < 0 || c >= ncols) f |= 2;
      if (c <= prev) f |= 4;
      if (noself && c == r) f |= 8;
      prev = c;
    }
    if (f) atomicOr(flag, f);
  }
}

__global__ void k_maxlen(const int* rowptr, long long nrows, int* out) {
  int m = 0;
  FSDA_GRID_LOOP(r, nrows) m = max(m, rowptr[r + 1] - rowptr[r]);
  atomicMax(out, m);
}

// histogram of column indices
__global__ void k_col_count(const int* col, long long nnz, int* cnt) { FSDA_GRID_LOOP(k, nnz) atomicAdd(&cnt[col[k]], 1); }

// cnt[0] positives, cnt[1] negatives, cnt[2] error bits (1 range, 2 repeat, 4 label value).
__global__ void k_check_labels(const int* idx, const int8_t* y, long long nl, long long n, int* mark, int* cnt) {
  FSDA_GRID_LOOP(k, nl) {
    const int i = idx[k];
    if (i < 0 || i >= n) {
      atomicOr(&cnt[2], 1);
      continue;
    }
    if (atomicAdd(&mark[i], 1) != 0) atomicOr(&cnt[2], 2);
    const int yy = y[k];
    if (yy == 1)
      atomicAdd(&cnt[0], 1);
    else if (yy == -1)
      atomicAdd(&cnt[1], 1);
    else
      atomicOr(&cnt[2], 4);
  }
}

// labw = 1/l on labeled rows (mean weight), ycen = y - mean(y), zw = +1/N+ or -1/N-.
__global__ void k_label_vectors(const int* idx, const int8_t* y, long long nl, int npos, int nneg, double* labw,
                                double* ycen, double* zw) {
  const double l = (double)nl;
  const double ybar = (double)(npos - nneg) / l;
  FSDA_GRID_LOOP(k, nl) {
    const int i = idx[k];
    const bool pos = y[k] > 0;
    labw[i] = 1.0 / l;
    ycen[i] = (pos ? 1.0 : -1.0) - ybar;
    zw[i] = pos ? 1.0 / (double)npos : -1.0 / (double)nneg;
  }
}

__global__ void k_tile_rows(const int* rowptr, int nrows, long long nnz, int ntiles, int tile, int* tile_row) {
  FSDA_GRID_LOOP(b, (long long)ntiles + 1) {
    if (b == ntiles) {
      tile_row[b] = nrows;
      continue;
    }
    const long long target = b * (long long)tile;
    int lo = 0, hi = nrows;  // first r in [0, nrows] with rowptr[r] >= target
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((long long)rowptr[mid] >= target) hi = mid; else lo = mid + 1;
    }
    tile_row[b] = lo;
  }
}

__global__ void k_cross(const int* rowptr, long long nnz, int ntiles, int tile, const int* tile_row, int* cross) {
  FSDA_GRID_LOOP(b, ntiles) {
    const int r0 = tile_row[b], r1 = tile_row[b + 1];
    const long long hi = min((b + 1) * (long long)tile, nnz);
    cross[b] = (r1 > r0 && (long long)rowptr[r1] > hi) ? r1 - 1 : -1;
  }
}

__global__ void k_expand_rows(const int* rowptr, long long nrows, int* rowid) {
  FSDA_GRID_LOOP(r, nrows) for (int k = rowptr[r]; k < rowptr[r + 1]; k++) rowid[k] = (int)r;
}

// rowptr[j] = first position of key >= j in the sorted key array.
__global__ void k_keys_to_rowptr(const int* keys, long long nnz, int ncols, int* rowptr) {
  FSDA_GRID_LOOP(j, (long long)ncols + 1) {
    long long lo = 0, hi = nnz;
    while (lo < hi) {
      const long long mid = (lo + hi) >> 1;
      if (keys[mid] >= j) hi = mid; else lo = mid + 1;
    }
    rowptr[j] = (int)lo;
  }
}

// For the row lengths len[0..n) in decreasing order: out[k] = number of rows
// with length >= thr[k] (k < nthr).
__global__ void k_count_at_least(const int* len, long long n, const int* thr, int nthr, int* out) {
  const int k = threadIdx.x;
  if (k >= nthr) return;
  long long lo = 0, hi = n;  // first index with len < thr
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (len[mid] >= thr[k]) lo = mid + 1; else hi = mid;
  }
  out[k] = (int)lo;
}

}  // namespace fsda
