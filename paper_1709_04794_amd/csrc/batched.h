// Batched conjugate gradients: T right-hand sides ("columns") against one SDA
// operator, column c solving (X^T M' X + sigma_c I) x_c = b_c with its own
// shift.  The three sparse products are applied to all T columns at once, so
// every index is read once per iteration for the whole batch.
//
// Used for the correction solves of the mixed-precision path: the FP64
// residuals R_s = b - A(beta_s) w_s of different shifts are not collinear, so
// they cannot share one shifted Krylov basis and are solved as independent
// systems (one column per shift), in FP32.
//
// Layout: vectors are column-interleaved, element (row j, column c) at
// j * T + c.  A group of T lanes owns one row: the gather of one nonzero
// fetches T contiguous FP32 values, and the group shares the index load.
// Vectors and sparse sums are FP32; dot products and the per-column CG scalars
// are FP64.  Reductions: every producing block writes one FP64 partial per
// column; a one-block kernel sums them in a fixed order and updates the
// per-column scalars, which the next kernels read.  No device-scope fence.
#pragma once

#include "kernels.h"

namespace fsda {

constexpr int BT_MAX = 64;  // columns of a batch
constexpr int BU = 8;       // nonzeros in flight per lane

struct BState {
  int iter, stop, status, maxit;
  int ncol, zero, pad_[2];       // zero: always 0, the stop flag of launches outside the recurrence
  double trel;                   // relative stop floor (of ||b_c||)
  double rr[BT_MAX];             // <r_c, r_c>
  double a[BT_MAX], b[BT_MAX];   // CG step and direction coefficients of the iteration
  double tabs[BT_MAX];           // absolute stop target per column
  double tol[BT_MAX];            // max(tabs, trel ||b_c||)
  double bnorm[BT_MAX];
  double sigma[BT_MAX];          // shift of column c
  double cm[BT_MAX];             // labeled mean of t_c (centring)
  int active[BT_MAX];
  int conv[BT_MAX];              // iterations after which column c stopped
  double res2[BT_MAX];           // true residual ||b_c - A(sigma_c) x_c||^2 after a solve
};

// Per-column block sum of acc (thread tid holds column tid % T) into
// part[blockIdx.x * T + c], summed over the groups in a fixed order.
template <int T, int NT = BS>
__device__ __forceinline__ void write_partials_cols(double* part, double acc) {
  __shared__ double sh[NT];
  constexpr int G = NT / T;
  const int tid = threadIdx.x;
  __syncthreads();
  sh[tid] = acc;
  __syncthreads();
  if (tid < T) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < G; k++) t += sh[k * T + tid];
    part[(size_t)blockIdx.x * T + tid] = t;
  }
}

// The same into slot `slot` (part[slot * T + c]).
template <int T>
__device__ __forceinline__ void write_partials_cols_at(double* part, int slot, double acc) {
  __shared__ double sh[BS];
  constexpr int G = BS / T;
  const int tid = threadIdx.x;
  __syncthreads();
  sh[tid] = acc;
  __syncthreads();
  if (tid < T) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < G; k++) t += sh[k * T + tid];
    part[(size_t)slot * T + tid] = t;
  }
}

// The same into slot `slot` for partials held column by column in runs of RB
// threads (thread t < RB T holds column t / RB; the others hold nothing).
template <int T, int RB>
__device__ __forceinline__ void write_partials_rows(double* part, int slot, double acc) {
  __shared__ double sh[BS];
  const int tid = threadIdx.x;
  __syncthreads();
  sh[tid] = acc;
  __syncthreads();
  if (tid < T) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < RB; k++) t += sh[tid * RB + k];
    part[(size_t)slot * T + tid] = t;
  }
}

// out[c] (shared memory, c < T) = sum over blocks of part[blk * T + c], in a
// fixed order.  All threads of the block must call it.
template <int T, int NT = BS>
__device__ void col_sums(const double* part, int nblk, double* out) {
  __shared__ double sh[NT];
  constexpr int G = NT / T;
  constexpr int U = 32;  // loads in flight per thread: a few thousand partials take a few round trips
  const int c = threadIdx.x % T, g = threadIdx.x / T;
  double v = 0.0;
  for (int b0 = g; b0 < nblk; b0 += G * U) {
    double x[U];
#pragma unroll
    for (int u = 0; u < U; u++) x[u] = b0 + u * G < nblk ? part[(size_t)(b0 + u * G) * T + c] : 0.0;
#pragma unroll
    for (int u = 0; u < U; u++) v += x[u];
  }
  __syncthreads();
  sh[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < T) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < G; k++) t += sh[k * T + threadIdx.x];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// products over T columns: one group of T lanes per row, lane c = column c
// ---------------------------------------------------------------------------

// The labeled weights of row r for column c are w[r * ws + c * cs]: one
// labeled set for every column (ws = 1, cs = 0) or one per column (ws = T,
// cs = 1, interleaved like the vectors).

// t = X p; with W, partials of sum_r w_rc t_rc (w = 1/l on labeled rows).
template <int T, typename V, bool W>
struct BEpiX {
  using VT = V;
  V* t;
  const double* w;
  int ws, cs;
  static constexpr bool kReduce = W;
  __device__ void prepare(const double*, int) {}
  __device__ double row(int r, int c, V v) const {
    t[(size_t)r * T + c] = v;
    return W ? w[(size_t)r * ws + c * cs] * (double)v : 0.0;
  }
};

// u = M' t per column (the centring of each column with its own labeled mean
// cm_c); partials of <t_c, u_c>.
template <int T, typename V, bool LAB>
struct BEpiLap {
  using VT = V;
  const V* t;
  const double* labw;
  int ws, cs;
  const int* srowptr;
  V* u;
  double alpha;
  V cm;
  static constexpr bool kReduce = true;
  __device__ void prepare(const double* cmv, int c) { cm = LAB ? (V)cmv[c] : (V)0; }
  __device__ double row(int r, int c, V v) const {
    const V tr = t[(size_t)r * T + c];
    const V deg = (V)(srowptr[r + 1] - srowptr[r]);
    V x = (V)alpha * (deg * tr - v);
    if (LAB && labw[(size_t)r * ws + c * cs] != 0.0) x += (V)(1.0 - alpha) * (tr - cm);
    u[(size_t)r * T + c] = x;
    return (double)tr * (double)x;
  }
};

// Index registers per lane of a group's cooperative index load: a pass over a
// row reads T * BM(T) = 64 consecutive indices with one coalesced load per
// lane, then broadcasts them inside the group.
template <int T>
constexpr int BM() {
  return T >= 64 ? 1 : 64 / T;
}
// Nonzeros of one X^T chunk: one cooperative pass of every group of a block.
template <int T>
constexpr int BCHUNK() {
  return (BS / T) * T * BM<T>();
}
constexpr int BMED = 64;  // X^T rows shorter than this always get one group per row in the batched product

// Sum over the nonzeros [beg, end) of a row of src[col[k] * T + c] for the
// group's column c.  Lane c of the group loads the indices beg + m*T + c; each
// index then comes from its lane by a shuffle inside the group (all lanes of a
// group share the trip count, so every source lane is active), and the gathers
// of a pass are independent of each other.
// With GPR groups per row, group `sub` of a row takes the passes sub, sub +
// GPR, ... (the caller adds the GPR groups' sums).
template <int T, typename V, int GPR = 1>
__device__ __forceinline__ V group_gather(const int* __restrict__ col, int beg, int end, const V* __restrict__ src,
                                          int c, int sub = 0) {
  constexpr int M = BM<T>();
  V v = (V)0;
  for (int base = beg + sub * T * M; base < end; base += GPR * T * M) {
    int id[M];
#pragma unroll
    for (int m = 0; m < M; m++) {
      const int k = base + m * T + c;
      id[m] = k < end ? col[k] : -1;
    }
#pragma unroll
    for (int m = 0; m < M; m++) {
      if (base + m * T >= end) break;  // uniform over the group
#pragma unroll
      for (int q = 0; q < T; q++) {
        const int idx = __shfl(id[m], q, T);
        v += idx >= 0 ? src[(size_t)idx * T + c] : (V)0;
      }
    }
  }
  return v;
}

// The X product over T columns reads its most frequent features, the mask
// features [0, nmask) (one 64-bit mask per row; the CSR then holds only the
// others), from a per-block shared copy of their T columns.
struct BMask {
  const unsigned long long* mask;
  int nmask;
};

// The GPR groups of one row (lanes g0 T .. (g0 + GPR) T - 1, g0 a multiple of
// GPR) add their sums: every lane c of them gets the row's column c.
template <int T, int GPR, typename V>
__device__ __forceinline__ V groups_sum(V v) {
#pragma unroll
  for (int o = T; o < T * GPR; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Rows of one CSR over T columns, GPR groups of T lanes per row (64 / (T GPR)
// rows per wave); `stop` (the solver's stop flag) ends the launch at once when
// set, cm holds the per-column labeled means.  With MASK, bm gives the masks
// and the launch has nmask * T values of V of dynamic shared memory.
template <int T, class Epi, bool MASK = false, int GPR = 1, int NT = BS>
__global__ __launch_bounds__(NT) void bk_rows(const int* __restrict__ rowptr, const int* __restrict__ col, int nrows,
                                              const typename Epi::VT* __restrict__ src, Epi epi, const int* stop,
                                              const double* cm, double* part, BMask bm) {
  using V = typename Epi::VT;
  if (*stop) return;
  constexpr int G = NT / T;
  constexpr int RB = G / GPR;  // rows per block and pass
  const int c = threadIdx.x % T, g = threadIdx.x / T, q = g % GPR;
  extern __shared__ double bk_smem[];
  V* hot = reinterpret_cast<V*>(bk_smem);
  if (MASK) {
    stage_lds<NT, 4>(hot, src, bm.nmask * T);
    __syncthreads();
  }
  epi.prepare(cm, c);
  double acc = 0.0;
  for (int r0 = blockIdx.x * RB; r0 < nrows; r0 += gridDim.x * RB) {
    const int r = r0 + g / GPR;  // the same for the GPR groups of a row
    if (r >= nrows) continue;
    V v = group_gather<T, V, GPR>(col, rowptr[r], rowptr[r + 1], src, c, q);
    if (MASK && q == 0) {
      unsigned long long mb = bm.mask[r];
      while (mb) {
        v += hot[(__ffsll((long long)mb) - 1) * T + c];
        mb &= mb - 1;
      }
    }
    v = groups_sum<T, GPR>(v);
    if (q == 0) acc += epi.row(r, c, v);
  }
  if (Epi::kReduce) write_partials_cols<T, NT>(part, acc);
}

// X^T product, first level.  Block items: the chunks of BCHUNK<T>() nonzeros
// of the rows [0, nmed) (each group sums its own slice of T * BM indices; the
// groups are added in a fixed order into lpart[chunk * T + c]); then the rows
// [nmed, d), one group per row: Q = X^T u + sigma_c P (P interleaved, or NULL
// for Q = X^T u).  Q is interleaved (ldq == 0: Q[r * T + c]) or column-major
// (Q[c * ldq + r]).
struct BXtArgs {
  const int* rowptr;
  const int* col;
  int d, nmed, nchunk;
  const int* chunk_row;
  const int* chunk_beg;
  const int* row_chunk0;
  // XCD slices (item_chunk != NULL): a row of >= BMED nonzeros is cut at the
  // sample boundaries x n / 8 as well, chunk k ending at chunk_end[k], and
  // chunk item it (of nitem, a multiple of 8) sums chunk item_chunk[it] (-1:
  // none), a chunk of sample slice it % 8: with a grid that is a multiple of 8
  // every XCD gathers from one eighth of u, which stays in its L2.
  const int* chunk_end;
  const int* item_chunk;
  int nitem;
  // chunk k's sum goes to lpart[(part0 + k) T + c]; the first part0 pieces are
  // the LDS-slice parts of the longest rows (BXtLds), rows [0, part0 / nslice)
  int part0;
};

// LDS slices of the batched X^T product.  The longest rows of X^T [0, nrow) (at
// least BL_SEG nonzeros per slice on average) are summed per slice of slen
// samples from u over those samples and the T columns, staged in LDS
// (slen T values, 128 KiB in FP64): gathers from LDS pay no cache-line lookups
// and move no L2 bytes.  Part (row j, slice x) goes to lpart[(j nslice + x) T
// + c], which bk_xt_rows adds in slice order.  The rows' indices are copied
// slice-major as 16-bit offsets in the slice, each segment at a multiple of
// LVEC entries and padded to one with the offset slen (a zero row of LDS).
constexpr int BLT = 1024;                  // threads per block of bk_xt_lds
constexpr int BL_LDS_BYTES = 128 * 1024;   // staged slice of u (one block per CU)
constexpr int BL_SEG = 16;                 // shortest average segment of a row taken
constexpr int BLX = 8;                     // index loads per group and pass

struct BXtLds {
  int nslice, slen, n, nrow;  // slices of slen samples; rows [0, nrow) of X^T
  int nitem, nblk;            // items per slice (BLT / T rows each); blocks
  const int* xptr;            // [nslice][nrow + 1]: segment starts (multiples of LVEC)
  const unsigned short* xcol; // slice-major offsets, padded with slen
};

__device__ __forceinline__ size_t qidx(int T, long long ldq, long long r, int c) {
  return ldq ? (size_t)c * ldq + r : (size_t)r * T + c;
}

// The residual update fused into the X^T product of the target batch (ring !=
// NULL): instead of storing q, the product's epilogue writes r_{i+1} = r_i -
// a_c q to ring slot (i + 1) mod m (r_i in slot i mod m, i = *iter; the ring is
// column-major like Q, [slot][c][row] with row stride ld) and adds r_{i+1}^2 to
// the block's per-column partials, stored in slot slot0 + block of part.
struct BResid {
  const int* iter;
  int m;
  double* ring;
  long long ld;
  const double* a;
  double* part;
  int slot0;
};

// The same for the batched column solves (kernels instantiated with CU), whose
// vectors are all interleaved: the product's epilogue does r = R - a_c q, R = r, X += a_c P
// (P the product's direction) instead of storing q, with the per-column
// partials of <r, r> in slot slot0 + block of part.
template <typename V>
struct BColResid {
  V* R;
  V* X;
  const double* a;
  double* part;
  int slot0;
};

template <int T, typename V, int GPR = 1, bool CU = false>
__global__ __launch_bounds__(BS) void bk_xt(BXtArgs X, V* lpart, const V* __restrict__ u, const V* __restrict__ P,
                                            V* Q, long long ldq, const double* sigma, const int* stop,
                                            BResid R = BResid{nullptr, 0, nullptr, 0, nullptr, nullptr, 0},
                                            BColResid<V> CR = BColResid<V>{nullptr, nullptr, nullptr, nullptr, 0}) {
  if (*stop) return;
  double acc = 0.0;  // fused residual update: this block's <r_{i+1}, r_{i+1}> for the lane's column
  const double* rin = nullptr;
  double* rout = nullptr;
  if (R.ring) {
    const int i = *R.iter;
    rin = R.ring + (size_t)(i % R.m) * T * R.ld;
    rout = R.ring + (size_t)((i + 1) % R.m) * T * R.ld;
  }
  const int* __restrict__ rowptr = X.rowptr;
  const int* __restrict__ col = X.col;
  const int d = X.d, nmed = X.nmed, nchunk = X.nchunk;
  const int* __restrict__ chunk_row = X.chunk_row;
  const int* __restrict__ chunk_beg = X.chunk_beg;
  constexpr int G = BS / T;
  constexpr int SL = T * BM<T>();  // nonzeros of a group's slice
  __shared__ V sh[BS];
  constexpr int RB = G / GPR;  // short rows per item
  __shared__ double tq[T * (RB + 1)];
  const int c = threadIdx.x % T, g = threadIdx.x / T;
  const V sg = P ? (V)sigma[c] : (V)0;
  const int q = g % GPR;
  const int nchit = X.item_chunk ? X.nitem : nchunk;  // chunk items
  const int nitems = nchit + (d - nmed + RB - 1) / RB;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    if (it < nchit) {  // uniform over the block
      const int k = X.item_chunk ? X.item_chunk[it] : it;
      if (k < 0) continue;
      const int r = chunk_row[k];
      const int end = X.chunk_end ? X.chunk_end[k] : rowptr[r + 1];
      const int beg = min(chunk_beg[k] + g * SL, end);
      const V v = group_gather<T, V>(col, beg, min(beg + SL, end), u, c);
      __syncthreads();
      sh[threadIdx.x] = v;
      __syncthreads();
      if (threadIdx.x < T) {
        V t = (V)0;
#pragma unroll
        for (int q = 0; q < G; q++) t += sh[q * T + threadIdx.x];
        lpart[(size_t)(X.part0 + k) * T + threadIdx.x] = t;
      }
      continue;
    }
    const int r0 = nmed + (it - nchit) * RB;
    const int r = r0 + g / GPR;
    const bool live = r < d;
    V qv = (V)0;
    if (live) {
      const V v = groups_sum<T, GPR>(group_gather<T, V, GPR>(col, rowptr[r], rowptr[r + 1], u, c, q));
      qv = P ? v + sg * P[(size_t)r * T + c] : v;
    }
    if (rout) {
      // the item's RB x T results through LDS, so that the column-major ring is
      // read and written RB consecutive rows per column at a time
      if (live && q == 0) tq[c * (RB + 1) + g / GPR] = (double)qv;
      __syncthreads();
      if (threadIdx.x < RB * T) {
        const int cc = threadIdx.x / RB, jj = threadIdx.x % RB;
        if (r0 + jj < d) {
          const size_t e = (size_t)cc * R.ld + r0 + jj;
          const double x = rin[e] - R.a[cc] * tq[cc * (RB + 1) + jj];
          rout[e] = x;
          acc += x * x;  // column threadIdx.x / RB
        }
      }
      __syncthreads();
    } else if (CU) {
      if (live && q == 0) {
        const size_t e = (size_t)r * T + c;
        const double a = CR.a[c];
        const V x = (V)((double)CR.R[e] - a * (double)qv);
        CR.R[e] = x;
        CR.X[e] = (V)((double)CR.X[e] + a * (double)P[e]);
        acc += (double)x * (double)x;
      }
    } else if (live && q == 0) {
      Q[qidx(T, ldq, r, c)] = qv;
    }
  }
  if (R.ring) write_partials_rows<T, RB>(R.part, R.slot0 + blockIdx.x, acc);
  if (CU) write_partials_cols_at<T>(CR.part, CR.slot0 + blockIdx.x, acc);
}

// The LDS-slice parts (see BXtLds).  The (slice, item) work items, slice-major,
// are dealt to the blocks in contiguous ranges of equal size; a block stages u
// over each slice its range touches and takes that slice's items.  Group g (T
// lanes, lane c for column c) of an item sums row j's segment: the group's
// lanes load the same LVEC offsets (one 16-byte load, BLX in flight) and lane c
// adds lu[offset T + c] (T consecutive values: one LDS line per offset).
template <int T, typename V>
__global__ __launch_bounds__(BLT) void bk_xt_lds(BXtLds L, const V* __restrict__ u, V* lpart, const int* stop) {
  if (*stop) return;
  extern __shared__ double bl_raw[];
  V* lu = reinterpret_cast<V*>(bl_raw);  // (slen + 1) T values: the slice, then a zero row
  constexpr int G = BLT / T;
  const int c = threadIdx.x % T, g = threadIdx.x / T;
  const long long total = (long long)L.nslice * L.nitem;
  const int w0 = (int)(total * blockIdx.x / L.nblk), w1 = (int)(total * (blockIdx.x + 1) / L.nblk);
  const uint4* xv = reinterpret_cast<const uint4*>(L.xcol);
  const unsigned pad2 = (unsigned)L.slen | ((unsigned)L.slen << 16);
  for (int w = w0; w < w1;) {
    const int x = w / L.nitem;
    const int wend = min(w1, (x + 1) * L.nitem);
    __syncthreads();  // every group is done with the previous slice
    const long long s0 = (long long)x * L.slen;
    const int len = (int)min((long long)L.slen, (long long)L.n - s0) * T;
    stage_lds<BLT, 16>(lu, u + (size_t)s0 * T, len);
    if (threadIdx.x < T) lu[(size_t)L.slen * T + threadIdx.x] = (V)0;
    __syncthreads();
    const int* xp = L.xptr + (long long)x * (L.nrow + 1);
    for (int it = w - x * L.nitem; it < wend - x * L.nitem; it++) {
      const int j = it * G + g;
      if (j >= L.nrow) continue;
      V v = (V)0;
      const int ve = xp[j + 1] / LVEC;
      for (int k0 = xp[j] / LVEC; k0 < ve; k0 += BLX) {
        uint4 q[BLX];
#pragma unroll
        for (int e = 0; e < BLX; e++) q[e] = k0 + e < ve ? xv[k0 + e] : make_uint4(pad2, pad2, pad2, pad2);
#pragma unroll
        for (int e = 0; e < BLX; e++) {
          const unsigned wd[4] = {q[e].x, q[e].y, q[e].z, q[e].w};
#pragma unroll
          for (int h = 0; h < 4; h++)
            v += lu[(size_t)(wd[h] & 0xffffu) * T + c] + lu[(size_t)(wd[h] >> 16) * T + c];
        }
      }
      lpart[((size_t)j * L.nslice + x) * T + c] = v;
    }
    w = wend;
  }
}

// Slice-major copy of the LDS-slice rows' indices: thread (x, j) copies row j's
// segment of slice x ([segp[x nrow + j], segp[(x+1) nrow + j])) to
// xcol[xptr[x (nrow+1) + j] ..] as offsets from the slice's first sample, then
// fills the rest of its entries (up to the next segment's start) with slen.
__global__ __launch_bounds__(BS) void bk_slice_copy(const int* __restrict__ col, const int* __restrict__ segp,
                                                    const int* __restrict__ xptr, int nrow, int nslice, int slen,
                                                    unsigned short* xcol) {
  const long long t = (long long)blockIdx.x * BS + threadIdx.x;
  if (t >= (long long)nslice * nrow) return;
  const int x = (int)(t / nrow), j = (int)(t % nrow);
  const int b = segp[(long long)x * nrow + j], e = segp[(long long)(x + 1) * nrow + j];
  const int o = xptr[(long long)x * (nrow + 1) + j], o1 = xptr[(long long)x * (nrow + 1) + j + 1];
  const long long x0 = (long long)x * slen;
  for (int k = b; k < e; k++) xcol[o + (k - b)] = (unsigned short)(col[k] - x0);
  for (int k = o + (e - b); k < o1; k++) xcol[k] = (unsigned short)slen;
}

// X^T product, second level: row j < nmed is the fixed-order sum of its chunk
// sums lpart[row_chunk0[j] .. row_chunk0[j+1]) (the groups of a block take
// every G-th chunk, then add up in order), plus sigma_c P.
template <int T, typename V, bool CU = false>
__global__ __launch_bounds__(BS) void bk_xt_rows(BXtArgs X, const V* __restrict__ lpart, const V* __restrict__ P, V* Q,
                                                 long long ldq, const double* sigma, const int* stop,
                                                 BResid R = BResid{nullptr, 0, nullptr, 0, nullptr, nullptr, 0},
                                                 BColResid<V> CR = BColResid<V>{nullptr, nullptr, nullptr, nullptr, 0}) {
  if (*stop) return;
  double acc = 0.0;
  const double* rin = nullptr;
  double* rout = nullptr;
  if (R.ring) {
    const int i = *R.iter;
    rin = R.ring + (size_t)(i % R.m) * T * R.ld;
    rout = R.ring + (size_t)((i + 1) % R.m) * T * R.ld;
  }
  const int nmed = X.nmed;
  const int* __restrict__ row_chunk0 = X.row_chunk0;
  constexpr int G = BS / T;
  __shared__ V sh[BS];
  const int c = threadIdx.x % T, g = threadIdx.x / T;
  for (int j = blockIdx.x; j < nmed; j += gridDim.x) {
    const int c0 = row_chunk0[j], c1 = row_chunk0[j + 1];
    V v = (V)0;
    for (int k0 = c0 + g; k0 < c1; k0 += G * BU) {
      V x[BU];
#pragma unroll
      for (int e = 0; e < BU; e++) x[e] = k0 + e * G < c1 ? lpart[(size_t)(k0 + e * G) * T + c] : (V)0;
#pragma unroll
      for (int e = 0; e < BU; e++) v += x[e];
    }
    __syncthreads();
    sh[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < T) {
      const int cc = threadIdx.x;
      V t = (V)0;
#pragma unroll
      for (int k = 0; k < G; k++) t += sh[k * T + cc];
      const V qv = P ? t + (V)sigma[cc] * P[(size_t)j * T + cc] : t;
      if (rout) {
        const size_t e = (size_t)cc * R.ld + j;
        const double x = rin[e] - R.a[cc] * (double)qv;
        rout[e] = x;
        acc += x * x;
      } else if (CU) {
        const size_t e = (size_t)j * T + cc;
        const double a = CR.a[cc];
        const V x = (V)((double)CR.R[e] - a * (double)qv);
        CR.R[e] = x;
        CR.X[e] = (V)((double)CR.X[e] + a * (double)P[e]);
        acc += (double)x * (double)x;
      } else {
        Q[qidx(T, ldq, j, cc)] = qv;
      }
    }
  }
  if (R.ring) write_partials_cols_at<T>(R.part, R.slot0 + blockIdx.x, acc);
  if (CU) write_partials_cols_at<T>(CR.part, CR.slot0 + blockIdx.x, acc);
}

// ---------------------------------------------------------------------------
// batched CG recurrences
// ---------------------------------------------------------------------------

// R = P = B_c (rounded to V; zero for c >= ncol), X = 0; partials of <r, r>.
template <int T, typename V>
__global__ __launch_bounds__(BS) void bk_init(const double* __restrict__ B, long long ldb, int ncol, V* R, V* P, V* X,
                                              long long d, double* part) {
  constexpr int G = BS / T;
  const int c = threadIdx.x % T, g = threadIdx.x / T;
  double acc = 0.0;
  for (long long j = (long long)blockIdx.x * G + g; j < d; j += (long long)gridDim.x * G) {
    const V x = c < ncol ? (V)B[(long long)c * ldb + j] : (V)0;
    const size_t e = (size_t)j * T + c;
    R[e] = x;
    P[e] = x;
    X[e] = (V)0;
    acc += (double)x * (double)x;
  }
  write_partials_cols<T>(part, acc);
}

// rr_c, ||b_c||, tol_c; columns with a zero right-hand side, or one already
// within its target, never start.  One block.
template <int T>
__global__ __launch_bounds__(BS) void bk_init_done(BState* st, const double* part, int np) {
  __shared__ double rr[T];
  __shared__ int any;
  col_sums<T>(part, np, rr);
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  const int c = threadIdx.x;
  if (c < T) {
    const double bn = sqrt(rr[c]);
    const double tol = fmax(st->tabs[c], st->trel * bn);
    st->rr[c] = rr[c];
    st->bnorm[c] = bn;
    st->tol[c] = tol;
    st->conv[c] = 0;
    const int on = c < st->ncol && rr[c] > 0.0 && bn > tol;
    st->active[c] = on;
    if (on) atomicOr(&any, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0 && !any) st->stop = 1;
}

// out[c] = sum of the partials (one block; the labeled means of the X product).
template <int T>
__global__ __launch_bounds__(BS) void bk_colsum(const int* stop, const double* part, int np, double* out) {
  if (*stop) return;
  __shared__ double s[T];
  col_sums<T>(part, np, s);
  if (threadIdx.x < T) out[threadIdx.x] = s[threadIdx.x];
}

// a_c = <r,r>_c / (<t,u>_c + sigma_c <p,p>_c) for the active columns (0 for
// the others); a breakdown of an active column stops the solve.  One block.
template <int T>
__global__ __launch_bounds__(BS) void bk_step_a(BState* st, const double* tu_part, int ntu, const double* pp_part,
                                                int npp) {
  if (st->stop) return;
  __shared__ double tu[T], pp[T];
  __shared__ int bad;
  col_sums<T>(tu_part, ntu, tu);
  col_sums<T>(pp_part, npp, pp);
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const int c = threadIdx.x;
  if (c < T) {
    double a = 0.0;
    if (st->active[c]) {
      const double pq = tu[c] + st->sigma[c] * pp[c];
      a = st->rr[c] / pq;
      if (!(pq > 0.0) || !isfinite(a)) {
        atomicOr(&bad, 1);
        a = 0.0;
      }
    }
    st->a[c] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0 && bad) {
    st->status = FSDA_E_BREAKDOWN;
    st->stop = 1;
  }
}

// R -= a_c Q, X += a_c P; partials of <r, r>.
template <int T, typename V>
__global__ __launch_bounds__(BS) void bk_resid(const BState* st, const V* __restrict__ Q, const V* __restrict__ P, V* R,
                                               V* X, long long d, double* part) {
  if (st->stop) return;
  constexpr int G = BS / T;
  const int c = threadIdx.x % T, g = threadIdx.x / T;
  const double a = st->a[c];
  double acc = 0.0;
  for (long long j = (long long)blockIdx.x * G + g; j < d; j += (long long)gridDim.x * G) {
    const size_t e = (size_t)j * T + c;
    const V r = (V)((double)R[e] - a * (double)Q[e]);
    R[e] = r;
    X[e] = (V)((double)X[e] + a * (double)P[e]);
    acc += (double)r * (double)r;
  }
  write_partials_cols<T>(part, acc);
}

// rr' = <r,r>; b_c = rr'/rr_c; per-column stop test ||r_c|| <= tol_c; iteration
// count; stop when no column is active or at maxit.  One block.
template <int T>
__global__ __launch_bounds__(BS) void bk_step_b(BState* st, const double* rr_part, int nrr) {
  if (st->stop) return;
  __shared__ double rrn[T];
  __shared__ int any;
  col_sums<T>(rr_part, nrr, rrn);
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  const int i = st->iter;
  const int c = threadIdx.x;
  if (c < T) {
    double b = 0.0;
    if (st->active[c]) {
      b = rrn[c] / st->rr[c];
      st->rr[c] = rrn[c];
      st->conv[c] = i + 1;
      if (sqrt(rrn[c]) <= st->tol[c])
        st->active[c] = 0;
      else
        atomicOr(&any, 1);
    }
    st->b[c] = b;
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

// P = R + b_c P for the columns still active (the others keep P); partials of <p, p>.
template <int T, typename V>
__global__ __launch_bounds__(BS) void bk_pupdate(const BState* st, const V* __restrict__ R, V* P, long long d,
                                                 double* part) {
  if (st->stop) return;
  constexpr int G = BS / T;
  const int c = threadIdx.x % T, g = threadIdx.x / T;
  const double b = st->b[c];
  const bool on = st->active[c] != 0;
  double acc = 0.0;
  for (long long j = (long long)blockIdx.x * G + g; j < d; j += (long long)gridDim.x * G) {
    const size_t e = (size_t)j * T + c;
    V p = P[e];
    if (on) {
      p = (V)((double)R[e] + b * (double)p);
      P[e] = p;
    }
    acc += (double)p * (double)p;
  }
  write_partials_cols<T>(part, acc);
}

// W[c * ldw + j] += X[j * T + c] for c < ncol (FP64 accumulation of the correction).
template <int T, typename V>
__global__ __launch_bounds__(BS) void bk_add(const V* __restrict__ X, double* W, long long ldw, int ncol, long long d) {
  constexpr int G = BS / T;
  const int c = threadIdx.x % T, g = threadIdx.x / T;
  if (c >= ncol) return;
  for (long long j = (long long)blockIdx.x * G + g; j < d; j += (long long)gridDim.x * G)
    W[(long long)c * ldw + j] += (double)X[(size_t)j * T + c];
}

// partials of ||B_c - (Q + sigma_c X)_c||^2 (B column-major [c][ldb], Q and X
// interleaved): the true residual of A(sigma_c) x_c = b_c once Q = X^T M' X x.
template <int T, typename V>
__global__ __launch_bounds__(BS) void bk_resnorm(const BState* st, const double* __restrict__ B, long long ldb, int ncol,
                                                 const V* __restrict__ Q, const V* __restrict__ X, long long d,
                                                 double* part) {
  constexpr int G = BS / T;
  const int c = threadIdx.x % T, g = threadIdx.x / T;
  const double sg = st->sigma[c];
  double acc = 0.0;
  if (c < ncol)
    for (long long j = (long long)blockIdx.x * G + g; j < d; j += (long long)gridDim.x * G) {
      const size_t e = (size_t)j * T + c;
      const double r = B[(size_t)c * ldb + j] - ((double)Q[e] + sg * (double)X[e]);
      acc += r * r;
    }
  write_partials_cols<T>(part, acc);
}

// out[c * d + jj] = X[old2new[jj] * T + c] for c < ncol (interleaved, internal
// feature order -> one row per column in the caller's order).
template <int T, typename V>
__global__ void bk_unpack(const V* __restrict__ X, const int* __restrict__ old2new, double* out, int ncol, long long d) {
  FSDA_GRID_LOOP(e, (long long)ncol * d) {
    const long long c = e / d, jj = e % d;
    out[e] = (double)X[(size_t)old2new[jj] * T + c];
  }
}

// out[jj] = X[old2new[jj] * T + c] for one column c (into its own row of the caller's array).
template <int T, typename V>
__global__ void bk_unpack_col(const V* __restrict__ X, const int* __restrict__ old2new, double* out, int c,
                              long long d) {
  FSDA_GRID_LOOP(jj, d) out[jj] = (double)X[(size_t)old2new[jj] * T + c];
}

}  // namespace fsda
