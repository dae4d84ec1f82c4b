// Device code of the multi-shift SDA solver (gfx950, wave64).
//
// Everything on this path is bound by memory bandwidth or latency: the sparse
// products are gather-sums over int32 column indices of binary matrices (no
// multiplies), the rest are streaming vector updates and FP64 dot products.
// The one dense contraction of the method, the target batch's fold of buffered
// residuals into the per-shift state, runs on the matrix cores (targets.h).
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
constexpr int MAXS = 64;      // shifts per handle
constexpr int MAXCHUNK = 256;  // iterations per shift-state fold
constexpr int NPART = 4096;   // partials per reduction site
constexpr int MAXBIN = 8;     // row-length bins of a row product
constexpr int UNR = 8;        // independent loads per thread in streaming loops
constexpr int RUNR = 4;       // nonzeros per lane per pass in k_rows
constexpr int XUNR = 8;       // nonzeros per lane per pass in the X^T row bins

enum Site { SITE_X = 0, SITE_XT = 1, SITE_R = 2, SITE_TU = 3, SITE_PP = 4, NSITE = 5 };

// Last-block detection counts blocks in TG groups (block b in group b mod TG,
// each counter on its own 128-byte line) and then groups in one more counter:
// increments of a single address serialise at about 10 ns each, so one
// counter for 500 blocks would cost 5 us, the two levels about 0.5 us.
constexpr int TG = 16;
enum TicketSite { TK_STEP = 0, TK_DIR = 1, NTK = 2 };

// Solver state, resident in device memory.
struct State {
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
  double sigma0;           // seed shift of the shared recurrence
  double sig[MAXS];        // beta_s - sigma0
  double zp[MAXS], z[MAXS], zn[MAXS];  // zeta_{i-1}, zeta_i, zeta_{i+1}
  double as[MAXS], bs[MAXS];           // per-shift step and direction coefficients
  double res2[MAXS];       // ||b - A(beta_s) w_s||^2 after the solve
  int active[MAXS];
  int conv[MAXS];          // iteration at which shift s stopped
  double a_new, pq_new;    // a_i and <p_i, A p_i>, published by the X^T pass for the direction update
  alignas(128) unsigned int tk[NTK][TG + 1][32];  // last-block counters (one 128-byte line each)
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

// True in every thread of the last block to reach it.  Relaxed: the last
// block reads nothing the other blocks wrote in this kernel.  It also resets
// the counters, which no block touches any more, for the next launch.
__device__ __forceinline__ bool last_block(State* st, int site) {
  __shared__ int amlast;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int(*c)[32] = st->tk[site];
    const int ng = min(TG, (int)gridDim.x);
    const int g = blockIdx.x % ng;
    const unsigned int cnt = gridDim.x / ng + (g < (int)(gridDim.x % ng) ? 1u : 0u);
    int last = 0;
    if (atomicAdd(&c[g][0], 1u) == cnt - 1) last = atomicAdd(&c[TG][0], 1u) == (unsigned int)ng - 1;
    if (last) {
      for (int k = 0; k < ng; k++) c[k][0] = 0;
      c[TG][0] = 0;
    }
    amlast = last;
  }
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
    } else {  // identity step: w += 0 * P, P = 0 * r + 1 * P leave a frozen shift unchanged
      h[0] = 0.0;
      h[1] = 0.0;
      h[2] = 1.0;
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

// The shift state of thread s (shift s), loaded at the start of a kernel so
// that its last block can run step_scalars and resid_scalars on registers.
struct ShiftRegs {
  double zp, z, sig, a_prev, b_cur, tol;
  int active, nshift, maxit;
};
__device__ __forceinline__ ShiftRegs load_shift_regs(const State* st) {
  ShiftRegs q;
  q.nshift = st->nshift;
  q.maxit = st->maxit;
  q.a_prev = st->a_prev;
  q.b_cur = st->b_cur;
  q.tol = st->tol;
  const int s = threadIdx.x;
  q.active = 0;
  q.zp = q.z = q.sig = 0.0;
  if (s < q.nshift) {
    q.active = st->active[s];
    q.zp = st->zp[s];
    q.z = st->z[s];
    q.sig = st->sig[s];
  }
  return q;
}

// step_scalars(st, a) followed by resid_scalars(st, rrn, b, hist), the same
// arithmetic in the same order, from the registers q of the same kernel.
__device__ void step_resid_scalars(State* st, const ShiftRegs& q, int i, double a, double rrn, double b,
                                   double* hist) {
  const double rn = sqrt(rrn);
  const int slot = i % st->chunk;
  const int s = threadIdx.x;
  int still = 0;
  if (s < q.nshift) {
    double* h = hist + ((size_t)slot * MAXS + s) * 4;
    if (q.active) {
      const double den = a * q.b_cur * (q.zp - q.z) + q.zp * q.a_prev * (1.0 + q.sig * a);
      const double zn = q.zp * q.z * q.a_prev / den;
      const double as = a * zn / q.z;
      const double ratio = zn / q.z;
      const double bs = b * ratio * ratio;
      st->zn[s] = zn;
      st->as[s] = as;
      st->bs[s] = bs;
      h[0] = as;
      h[1] = zn;
      h[2] = bs;
      h[3] = 1.0;
      st->zp[s] = q.z;
      st->z[s] = zn;
      if (fabs(zn) * rn <= q.tol) {
        st->active[s] = 0;
        st->conv[s] = i + 1;
      } else {
        still = 1;
        if (i + 1 >= q.maxit) st->conv[s] = i + 1;
      }
    } else {  // identity step
      h[0] = 0.0;
      h[1] = 0.0;
      h[2] = 1.0;
      h[3] = 0.0;
    }
  }
  const int any = __syncthreads_or(still);
  if (threadIdx.x == 0) {
    st->a_cur = a;
    st->a_prev = a;
    st->b_cur = b;
    st->rr = rrn;
    st->iter = i + 1;
    if (!any) {
      st->stop = 1;
    } else if (i + 1 >= q.maxit) {
      st->stop = 1;
      st->status = FSDA_NOT_CONVERGED;
    }
  }
}

// ---------------------------------------------------------------------------
// row epilogues of the sparse products
// ---------------------------------------------------------------------------

// The epilogues are templated on the vector type V (double, or float on the
// mixed-precision path): row sums and vectors are V, reductions are double.

// t = X p; reduction <t, t> (the regression operator X^T X + sigma I, whose
// <p, A p> is <t, t> + sigma <p, p>).
template <typename T>
struct EpiXReg {
  using V = T;
  V* t;
  static constexpr bool kReduce = true;
  __device__ void prepare(const State*) {}
  __device__ double row(int r, V v) const {
    t[r] = v;
    return (double)v * (double)v;
  }
};

// t = X p; with W, reduction sum_r w_r t_r (w = 1/l on labeled rows gives their mean).
template <typename T, bool W>
struct EpiX {
  using V = T;
  V* t;
  const double* w;
  static constexpr bool kReduce = W;
  __device__ void prepare(const State*) {}
  __device__ double row(int r, V v) const {
    t[r] = v;
    return W ? w[r] * (double)v : 0.0;
  }
};

// u = M' t = (1-alpha)[r labeled](t_r - c) + alpha (d_r t_r - (S t)_r): the
// weight of Eq. SDAeig with the centring of Sec. 3.2.3 applied once, in sample
// space.  c (the labeled mean of t) is the sum of the X product's partials.
// Reduction <t, u> = p^T X^T M' X p, which with sigma <p, p> gives <p, A p>
// without a reduction over the X^T product.
template <typename T, bool LAB>
struct EpiLap {
  using V = T;
  const V* t;
  const double* labw;
  const int* srowptr;
  V* u;
  double alpha;
  const double* cpart;
  int ncpart;
  double c;
  static constexpr bool kReduce = true;  // <t, u> = <p, A p> - sigma <p, p>
  __device__ void prepare(const State*) { c = LAB ? sum_partials(cpart, ncpart) : 0.0; }
  __device__ double row(int r, V v) const {
    const V tr = t[r];
    const V deg = (V)(srowptr[r + 1] - srowptr[r]);
    V x = (V)alpha * (deg * tr - v);
    if (LAB && labw[r] != 0.0) x += (V)(1.0 - alpha) * (tr - (V)c);
    u[r] = x;
    return (double)tr * (double)x;
  }
};

// q = X^T u + sigma p (sigma read from *sigp when sigp is not NULL); reduction <p, q>.
template <typename T, bool RED>
struct EpiXT {
  using V = T;
  V* q;
  const V* p;
  double sigma;
  const double* sigp;
  static constexpr bool kReduce = RED;
  static constexpr bool kPublish = false;
  __device__ void prepare(const State*) {
    if (sigp) sigma = *sigp;
  }
  __device__ void publish(State*) const {}
  __device__ double row(int r, V v) const {
    const V pr = p ? p[r] : (V)0;
    const V qq = v + (V)sigma * pr;
    q[r] = qq;
    return (double)pr * (double)qq;
  }
};

// The step length of the shared recurrence, a_i = <r,r> / (<t,u> + sigma0 <p,p>),
// from the partials of the graph product and of the previous direction update
// (every block of a consumer sums them in the same order).
__device__ __forceinline__ double step_length(const State* st, const double* tu_part, int ntu, const double* pp_part,
                                              int npp, double* pq_out) {
  const double pq = sum_partials(tu_part, ntu) + st->sigma0 * sum_partials(pp_part, npp);
  *pq_out = pq;
  return st->rr / pq;
}

// X^T product fused with the residual update of the shared recurrence: for
// a row j of X^T, q_j = (X^T u)_j + sigma0 p_j and r_{i+1,j} = r_{i,j} - a_i q_j
// (ring slots i mod m and i+1 mod m); reduction <r_{i+1}, r_{i+1}>.  The long
// rows, left as chunk sums, are finished by the direction update (k_pupdate).
template <typename T>
struct EpiXTR {
  using V = T;
  const V* p;
  V* ring;
  long long ldd;
  const double* tu_part;
  int ntu;
  const double* pp_part;
  int npp;
  double a, sigma, pq;
  const V* rin;
  V* rout;
  static constexpr bool kReduce = true;
  static constexpr bool kPublish = true;  // a_i and <p, A p> for the direction update
  __device__ void publish(State* st) const {
    st->a_new = a;
    st->pq_new = pq;
  }
  __device__ void prepare(const State* st) {
    a = step_length(st, tu_part, ntu, pp_part, npp, &pq);
    sigma = st->sigma0;
    const int i = st->iter, m = st->chunk;
    rin = ring + (long long)(i % m) * ldd;
    rout = ring + (long long)((i + 1) % m) * ldd;
  }
  __device__ double row(int r, V v) const {
    const V q = v + (V)sigma * p[r];
    const V x = (V)((double)rin[r] - a * (double)q);
    rout[r] = x;
    return (double)x * (double)x;
  }
};

// True residual of one shift: R = b - (X^T u + beta w), stored when out is
// not NULL; reduction ||R||^2.
struct EpiRes {
  using V = double;
  const double* b;
  const double* w;
  double beta;
  double* out;
  static constexpr bool kReduce = true;
  static constexpr bool kPublish = false;
  __device__ void prepare(const State*) {}
  __device__ void publish(State*) const {}
  __device__ double row(int r, double v) const {
    const double R = b[r] - (v + beta * w[r]);
    if (out) out[r] = R;
    return R * R;
  }
};

// Spectral analysis (Alg. sasda) works in sample space with the identity in
// place of X: q = M' p + sigma p, where the centring uses the labeled mean of p
// (the sum of the partials the previous direction update wrote).  Reduction
// <p, M' p>, which with sigma <p, p> gives <p, q>.
struct EpiLapSA {
  using V = double;
  const double* p;
  const double* labw;
  const int* srowptr;
  double* q;
  double alpha, sigma;
  const double* cpart;
  int ncpart;
  double c;
  static constexpr bool kReduce = true;
  __device__ void prepare(const State* st) {
    c = sum_partials(cpart, ncpart);
    sigma = st->sigma0;
  }
  __device__ double row(int r, double v) const {
    const double pr = p[r];
    double x = alpha * ((double)(srowptr[r + 1] - srowptr[r]) * pr - v);
    if (labw[r] != 0.0) x += (1.0 - alpha) * (pr - c);
    q[r] = x + sigma * pr;
    return pr * x;
  }
};

// True residual of one shift of the spectral-analysis system:
// R = g - (M' z + beta z); reduction ||R||^2.
struct EpiResSA {
  using V = double;
  const double* g;
  const double* z;
  const double* labw;
  const int* srowptr;
  double alpha, beta;
  const double* cpart;
  int ncpart;
  double c;
  static constexpr bool kReduce = true;
  __device__ void prepare(const State*) { c = sum_partials(cpart, ncpart); }
  __device__ double row(int r, double v) const {
    const double zr = z[r];
    double x = alpha * ((double)(srowptr[r + 1] - srowptr[r]) * zr - v);
    if (labw[r] != 0.0) x += (1.0 - alpha) * (zr - c);
    const double R = g[r] - (x + beta * zr);
    return R * R;
  }
};

// partials of sum_j w_j v_j (the labeled mean when w = 1/l on labeled rows)
__global__ __launch_bounds__(BS) void k_wsum(const double* __restrict__ w, const double* __restrict__ v, long long n,
                                             double* part) {
  double acc = 0.0;
  for (long long j = (long long)blockIdx.x * BS + threadIdx.x; j < n; j += (long long)gridDim.x * BS)
    acc += w[j] * v[j];
  write_partial(part, blockIdx.x, acc);
}

// ---------------------------------------------------------------------------
// hold-out loss and hypergradient terms
// ---------------------------------------------------------------------------

// flag bits: 1 held-out index out of range, 2 repeated (mark: n zeroed counters)
__global__ void k_ho_check(const int* idx, long long nho, long long n, int* mark, int* flag) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nho; k += (long long)gridDim.x * blockDim.x) {
    const int i = idx[k];
    if (i < 0 || i >= n) {
      atomicOr(flag, 1);
      continue;
    }
    if (atomicAdd(&mark[i], 1) != 0) atomicOr(flag, 2);
  }
}

// e_k = t[idx_k] - y_k: v[idx_k] = e_k / n_ho (v zero elsewhere); partials of sum e_k^2.
__global__ __launch_bounds__(BS) void k_ho_resid(const double* __restrict__ t, const int* __restrict__ idx,
                                                 const double* __restrict__ y, long long nho, double* v,
                                                 double* part) {
  double acc = 0.0;
  for (long long k = (long long)blockIdx.x * BS + threadIdx.x; k < nho; k += (long long)gridDim.x * BS) {
    const double e = t[idx[k]] - y[k];
    v[idx[k]] = e / (double)nho;
    acc += e * e;
  }
  write_partial(part, blockIdx.x, acc);
}

// partials of <a, b>
__global__ __launch_bounds__(BS) void k_dot(const double* __restrict__ a, const double* __restrict__ b, long long n,
                                            double* part) {
  double acc = 0.0;
  for (long long j = (long long)blockIdx.x * BS + threadIdx.x; j < n; j += (long long)gridDim.x * BS) acc += a[j] * b[j];
  write_partial(part, blockIdx.x, acc);
}

// partials of sum w a b, sum w a, sum w b (w = 1/l on labeled rows)
__global__ __launch_bounds__(BS) void k_labdots(const double* __restrict__ w, const double* __restrict__ a,
                                                const double* __restrict__ b, long long n, double* p0, double* p1,
                                                double* p2) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (long long j = (long long)blockIdx.x * BS + threadIdx.x; j < n; j += (long long)gridDim.x * BS) {
    const double wj = w[j];
    s0 += wj * a[j] * b[j];
    s1 += wj * a[j];
    s2 += wj * b[j];
  }
  write_partial(p0, blockIdx.x, s0);
  write_partial(p1, blockIdx.x, s1);
  write_partial(p2, blockIdx.x, s2);
}

// partials of sum a_i b_i, sum a_i, sum b_i over the samples i = idx[k],
// k in [k0, k1) (one target's labeled set)
__global__ __launch_bounds__(BS) void k_idxdots(const int* __restrict__ idx, long long k0, long long k1,
                                                const double* __restrict__ a, const double* __restrict__ b,
                                                double* p0, double* p1, double* p2) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (long long k = k0 + (long long)blockIdx.x * BS + threadIdx.x; k < k1; k += (long long)gridDim.x * BS) {
    const int i = idx[k];
    s0 += a[i] * b[i];
    s1 += a[i];
    s2 += b[i];
  }
  write_partial(p0, blockIdx.x, s0);
  write_partial(p1, blockIdx.x, s1);
  write_partial(p2, blockIdx.x, s2);
}

// Rows of S over src = t_w: reduction <t_l, L t_w>, (L t_w)_r = d_r t_w,r - (S t_w)_r.
struct EpiLapDot {
  using V = double;
  const double* tw;
  const double* tl;
  const int* srowptr;
  static constexpr bool kReduce = true;
  __device__ void prepare(const State*) {}
  __device__ double row(int r, double v) const {
    return tl[r] * ((double)(srowptr[r + 1] - srowptr[r]) * tw[r] - v);
  }
};

// ---------------------------------------------------------------------------
// sparse products, lanes per row
// ---------------------------------------------------------------------------
//
// Rows are grouped in bins of similar length (for X^T the features are
// relabeled by decreasing frequency, so the bins are contiguous row ranges).
// In a bin, `lpr` lanes share a row and take RUNR nonzeros each per pass: all
// index loads, then all gathers, are in flight together; the lanes then add up
// with shuffles.  lpr == 0 marks rows known to be empty.

// In the X product the most frequent features (internal ids [0, MK), the
// relabeling puts them first) are held per sample as one 64-bit mask instead of
// CSR entries: their values are staged in shared memory and added per set bit,
// with no gathers.  The next most frequent ones, up to HOT, stay CSR entries
// but are read from the same shared copy: random 8-byte gathers are limited by
// the rate of distinct cache-line lookups, which shared memory does not pay.
constexpr int MK = 64;     // features in the mask
constexpr int HOT = 8192;  // features staged in shared memory by the X product (64 KiB of FP64)
constexpr int XNT = 1024;  // threads per block of the X product (two blocks and their copies fit a CU's LDS)
constexpr int HOT_REG = 2048;  // features staged by the regression phase's X product (blocks of BS threads)

struct Rows {
  const int* rowptr;
  const int* col;
  int nb;
  int row0[MAXBIN + 1];
  int lpr[MAXBIN];
  int item0[MAXBIN + 1];  // work items before bin b; an item is BS/lpr rows (BS when lpr == 0)
  const unsigned long long* mask;  // NULL, or per row the mask features (col then holds only the others)
  int mtop;                        // features in the mask, <= MK
  int nhot;                        // with mask: features [0, nhot) staged in shared memory, mtop <= nhot <= HOT
};

// Block sum over NT threads in a fixed order; every thread gets the result.
template <int NT>
__device__ __forceinline__ double block_sum_nt(double v) {
  __shared__ double sh[NT / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; i++) t += sh[i];
  return t;
}

// dst[k] = src[k] for k < len by the NT threads of a block, SU loads per thread
// in flight before their values are stored (a plain loop waits for each load
// before its store: one memory round trip per element a thread copies).
template <int NT, int SU, typename V>
__device__ __forceinline__ void stage_lds(V* dst, const V* __restrict__ src, int len) {
  for (int k0 = threadIdx.x; k0 < len; k0 += NT * SU) {
    V v[SU];
#pragma unroll
    for (int e = 0; e < SU; e++) {
      const int k = k0 + e * NT;
      v[e] = k < len ? src[k] : (V)0;
    }
#pragma unroll
    for (int e = 0; e < SU; e++) {
      const int k = k0 + e * NT;
      if (k < len) dst[k] = v[e];
    }
  }
}

// Row products in blocks of NT threads (an item is NT / lpr rows; the host plan
// is built for the same NT).
template <class Epi, int NT = BS>
__global__ __launch_bounds__(NT) void k_rows(Rows R, const typename Epi::V* __restrict__ src, Epi epi, State* st,
                                             double* part, int slot0, int solve) {
  using V = typename Epi::V;
  if (solve && st->stop) return;
  epi.prepare(st);
  const int tid = threadIdx.x;
  extern __shared__ double rows_smem[];  // with mask: src over the features [0, nhot), launched with that size
  V* ptop = reinterpret_cast<V*>(rows_smem);
  const int nhot = R.mask ? R.nhot : 0;
  if (R.mask) {
    stage_lds<NT, 8>(ptop, src, nhot);
    __syncthreads();
  }
  double acc = 0.0;
  const int nitems = R.item0[R.nb];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    int b = 0;
    while (it >= R.item0[b + 1]) b++;
    const int lpr = R.lpr[b];
    if (lpr == 0) {
      const int r = R.row0[b] + (it - R.item0[b]) * NT + tid;
      if (r < R.row0[b + 1]) acc += epi.row(r, (V)0);
      continue;
    }
    const int r = R.row0[b] + (it - R.item0[b]) * (NT / lpr) + tid / lpr;
    const int lane = tid & (lpr - 1);
    const bool live = r < R.row0[b + 1];
    V v = (V)0;
    if (live) {
      const int beg = R.rowptr[r], end = R.rowptr[r + 1];
      unsigned long long mine = 0;
      int mbase = 0;
      if (R.mask) {  // lane takes MK/lpr consecutive mask bits of its row
        const int nbits = MK / lpr;
        mbase = lane * nbits;
        const unsigned long long m = R.mask[r] >> mbase;
        mine = nbits >= 64 ? m : (m & ((1ull << nbits) - 1));
      }
      for (int k0 = beg + lane; k0 < end; k0 += lpr * RUNR) {
        int idx[RUNR];
        V g[RUNR];
#pragma unroll
        for (int u = 0; u < RUNR; u++) {
          const int k = k0 + u * lpr;
          idx[u] = k < end ? R.col[k] : -1;
        }
#pragma unroll
        for (int u = 0; u < RUNR; u++) g[u] = idx[u] >= 0 ? (idx[u] < nhot ? ptop[idx[u]] : src[idx[u]]) : (V)0;
#pragma unroll
        for (int u = 0; u < RUNR; u++) v += g[u];
      }
      while (mine) {
        v += ptop[mbase + __ffsll((long long)mine) - 1];
        mine &= mine - 1;
      }
    }
    for (int o = lpr >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (live && lane == 0) acc += epi.row(r, v);
  }
  if (Epi::kReduce) {
    const double t = block_sum_nt<NT>(acc);
    if (tid == 0) part[slot0 + blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// X^T product: long rows in single-row chunks, the others in length bins
// ---------------------------------------------------------------------------
//
// With features relabeled by decreasing frequency, the rows of X^T are sorted
// by length.  Each long row is cut into chunks of CHUNK nonzeros; a block sums
// one chunk (coalesced index loads, independent gathers, block reduction).  A
// row of one chunk is finished there; the rows of several chunks (the prefix
// [0, nlong)) leave their chunk sums in lpart[chunk], and the consumer adds up
// a row's chunk sums in order (k_pupdate, or k_assemble).  The remaining
// rows go through the same lanes-per-row bins as k_rows, in the same launch.
// With XCD slices (below) the long rows are cut at sample boundaries too.

constexpr int CH = 4096;        // nonzeros per pass over a long-row chunk (16 per thread)
constexpr int NCP = 8;          // passes per chunk (2: 65.0, 4: 65.6, 8: 65.7 solves/s at mid)
constexpr int CHUNK = NCP * CH; // nonzeros of a long-row chunk

// XCD slices.  Work-groups are dispatched to the eight XCDs round robin, so with a
// grid that is a multiple of eight (or one item per block) item `it` runs on XCD
// it % 8.  When the sample-space vector is larger than an XCD's L2, the rows of at
// least XCD_SPLIT_ROW nonzeros (not in LDS slices) are cut at the sample boundaries
// x n / 8 and segment x of
// every such row is given to items with it % 8 == x: each XCD then gathers from one
// eighth of the vector, which stays in its L2.  A split row's sum is the ordered sum
// of its parts (k_assemble).
constexpr int NSLICE = 8;        // XCDs of the chip
constexpr int SPLIT_ROW = 64;    // rows at least this long are split into LDS slices
// Rows at least this long are split into XCD slices (the large workload's X^T
// pass: 16 -> 229.1 us per launch against 240.2 with 64, its assembly 13.2
// against 9.3; with 4, 258.4 and 28.8: below about two nonzeros per slice a
// part per slice costs more than the L2 saves).
constexpr int XCD_SPLIT_ROW = 16;
constexpr int SLICE_LONG = 8192; // split rows at least this long are summed in block chunks

struct XtSlices {
  int nb;                   // bins of split rows processed lanes-per-row (0: no such bins)
  int row0[MAXBIN + 1];
  int lpr[MAXBIN];
  int item0[MAXBIN + 1];    // items of one slice before bin b (each item runs for all slices)
  int r0;                   // first split row (0; with the LDS head rows of the hybrid plan, their count)
  int nsplit;               // split rows [r0, r0 + nsplit)
  int nlc;                  // [r0, nlc) are summed in the chunk items, [nlc, r0 + nsplit) in the bins
  const int* segp;          // [(NSLICE + 1) * nsplit]: slice x of row j is [segp[x*nsplit+j-r0], segp[(x+1)*nsplit+j-r0])
  int part0;                // lpart index of part 0 of row nlc; row j >= nlc has parts part0 + NSLICE (j - nlc) + x
};

// LDS slices.  When the sample range is cut into at most MAXLSLICE slices of
// LSLICE samples, one slice of u fits a work-group's LDS, and the split rows'
// segments of that slice are summed from there (k_xt_lds): gathers from LDS pay
// no cache-line lookups, which bind the gathers from L2.  The split rows'
// indices are copied slice-major (slice x: the segments of rows 0, 1, ... in
// order, as 16-bit offsets in the slice), so a slice's index stream is
// contiguous; every segment starts at a multiple of LVEC entries and is padded
// to one with the offset LSLICE, a slot of LDS that holds zero, so that a lane
// loads LVEC offsets with one 16-byte load.  Part (row j, slice x) goes to
// parts[x * nsplit + j]; the X^T pass adds a split row's parts in a fixed order
// (see ASM_ROWS) and runs the epilogue (assembly items, before its other items).
constexpr int LSLICE = 8192;   // samples per LDS slice (64 KiB of FP64)
constexpr int MAXLSLICE = 32;  // more slices: the XCD slices instead
constexpr int LTB = 1024;      // threads per block of k_xt_lds
constexpr int LVEC = 8;        // 16-bit offsets per index load (16 bytes)
constexpr int LXV = 2;         // index loads per lane per pass

struct XtLds {
  int nslice;               // 0: not in use
  int n;                    // samples
  int nsplit;               // split rows [0, nsplit)
  int nblk;                 // blocks; block k takes work items [k W / nblk, (k+1) W / nblk), W = nslice * nitem
  int nitem;                // items of one slice (item0[nb])
  const int* xptr;          // [nslice * (nsplit + 1)]: slice x, row j: xcol[xptr[x (nsplit+1) + j] ..], multiples of LVEC
  const unsigned short* xcol;  // slice-major offsets in the slice, segments padded with LSLICE
  double* parts;            // [nslice * nsplit]
  int nb;                   // bins of split rows, lanes per row from the expected segment length
  int row0[MAXBIN + 1];
  int lpr[MAXBIN];
  int item0[MAXBIN + 1];    // items (LTB / lpr rows) of one slice before bin b
};

// Rows per assembly item of the X^T pass: a split row's LDS-slice parts (up to
// MAXLSLICE, or one per LDS slice in the hybrid plan: 184 at large) are added by
// BS / ASM_ROWS groups of lanes, so that a lane has a few loads in flight rather
// than a serial walk over the slices (the large workload's X^T pass: 240.2 ->
// 221.1 us per launch against one row per thread).
constexpr int ASM_ROWS = 16;
__host__ __device__ inline int xt_asm_items(int nasm) {
  return ((nasm + ASM_ROWS - 1) / ASM_ROWS + NSLICE - 1) / NSLICE * NSLICE;
}

struct XtWork {
  const int* rowptr;
  const int* col;
  int nasm;                // with LDS slices: split rows [0, nasm) finished from their parts
  int nslice_asm;          // their parts per row
  const double* parts;     // [nslice_asm * nasm]
  int nchunk;              // chunks of the long rows, all processed before the bins
  int nchunk_multi;        // the first ones, of the rows of more than one part; a row of one
                           // chunk is finished where it is summed
  const int* chunk_row;    // [nchunk] row of each chunk
  const int* chunk_beg;    // [nchunk] first nonzero of each chunk
  const int* chunk_end;    // [nchunk] one past its last nonzero
  double* lpart;           // [parts] chunk and slice sums
  XtSlices sl;             // bins of the split rows (sliced mode)
  Rows rows;               // bins of the other rows
};

// Sum of src over the nonzeros [beg, end) of a row shared by lpr lanes (this lane's share).
template <typename V>
__device__ __forceinline__ V lane_row_sum(const int* __restrict__ col, const V* __restrict__ src, int beg, int end,
                                          int lane, int lpr) {
  V v = (V)0;
  for (int k0 = beg + lane; k0 < end; k0 += lpr * XUNR) {
    int idx[XUNR];
    V g[XUNR];
#pragma unroll
    for (int u = 0; u < XUNR; u++) {
      const int k = k0 + u * lpr;
      idx[u] = k < end ? col[k] : -1;
    }
#pragma unroll
    for (int u = 0; u < XUNR; u++) g[u] = idx[u] >= 0 ? src[idx[u]] : (V)0;
#pragma unroll
    for (int u = 0; u < XUNR; u++) v += g[u];
  }
  return v;
}

template <class Epi>
__global__ __launch_bounds__(BS) void k_xt(XtWork X, const typename Epi::V* __restrict__ src, Epi epi, State* st,
                                           double* part, int solve) {
  using V = typename Epi::V;
  if (solve && st->stop) return;
  epi.prepare(st);
  if (Epi::kPublish && blockIdx.x == 0 && threadIdx.x == 0) epi.publish(st);
  const int tid = threadIdx.x;
  double acc = 0.0;
  __shared__ double ash[BS];
  // assembly items (ASM_ROWS rows each) rounded up to a multiple of NSLICE, so
  // that the XCD-slice items after them keep item % 8 == slice (with a grid that
  // is a multiple of 8)
  const int nasm_items = xt_asm_items(X.nasm);
  const int nitems = nasm_items + X.nchunk + NSLICE * X.sl.item0[X.sl.nb] + X.rows.item0[X.rows.nb];
  for (int it0 = blockIdx.x; it0 < nitems; it0 += gridDim.x) {
    if (it0 < nasm_items) {
      // split rows from their LDS-slice parts: ASM_ROWS rows per item, group g of
      // the block's BS / ASM_ROWS groups adds the parts of slices g, g + BS /
      // ASM_ROWS, ... (consecutive rows in consecutive lanes), then the groups'
      // sums are added in group order
      const int j = it0 * ASM_ROWS + tid % ASM_ROWS, g = tid / ASM_ROWS;
      double v = 0.0;
      if (j < X.nasm)
        for (int x = g; x < X.nslice_asm; x += BS / ASM_ROWS) v += X.parts[(long long)x * X.nasm + j];
      __syncthreads();
      ash[tid] = v;
      __syncthreads();
      if (tid < ASM_ROWS && j < X.nasm) {
        double t = 0.0;
        for (int k = 0; k < BS / ASM_ROWS; k++) t += ash[k * ASM_ROWS + tid];
        acc += epi.row(j, (V)t);
      }
      continue;
    }
    const int it = it0 - nasm_items;
    if (it < X.nchunk) {
      const int r = X.chunk_row[it];
      const int beg0 = X.chunk_beg[it];
      const int end = X.chunk_end[it];
      constexpr int U = CH / BS;
      V v = (V)0;
      for (int beg = beg0; beg < end; beg += CH) {
        int idx[U];
        V g[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
          const int k = beg + u * BS + tid;
          idx[u] = k < end ? X.col[k] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; u++) g[u] = idx[u] >= 0 ? src[idx[u]] : (V)0;
#pragma unroll
        for (int u = 0; u < U; u++) v += g[u];
      }
      const double t = block_sum_all((double)v);
      if (tid == 0) {
        if (it < X.nchunk_multi)
          X.lpart[it] = t;
        else
          acc += epi.row(r, (V)t);  // the whole row
      }
      continue;
    }
    int ir = it - X.nchunk;
    const XtSlices& S = X.sl;
    if (ir < NSLICE * S.item0[S.nb]) {  // a bin item of the split rows, for slice x = it % 8
      const int k = ir / NSLICE, x = ir % NSLICE;
      int b = 0;
      while (k >= S.item0[b + 1]) b++;
      const int lpr = S.lpr[b];
      const int j = S.row0[b] + (k - S.item0[b]) * (BS / lpr) + tid / lpr;
      const int lane = tid & (lpr - 1);
      const bool live = j < S.row0[b + 1];
      V v = (V)0;
      if (live)
        v = lane_row_sum<V>(X.col, src, S.segp[x * S.nsplit + j - S.r0], S.segp[(x + 1) * S.nsplit + j - S.r0], lane,
                            lpr);
      for (int o = lpr >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (live && lane == 0) X.lpart[S.part0 + NSLICE * (j - S.nlc) + x] = (double)v;
      continue;
    }
    ir -= NSLICE * S.item0[S.nb];
    const Rows& R = X.rows;
    int b = 0;
    while (ir >= R.item0[b + 1]) b++;
    const int lpr = R.lpr[b];
    if (lpr == 0) {
      const int r = R.row0[b] + (ir - R.item0[b]) * BS + tid;
      if (r < R.row0[b + 1]) acc += epi.row(r, (V)0);
      continue;
    }
    const int r = R.row0[b] + (ir - R.item0[b]) * (BS / lpr) + tid / lpr;
    const int lane = tid & (lpr - 1);
    const bool live = r < R.row0[b + 1];
    V v = (V)0;
    if (live) v = lane_row_sum<V>(R.col, src, R.rowptr[r], R.rowptr[r + 1], lane, lpr);
    for (int o = lpr >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (live && lane == 0) acc += epi.row(r, v);
  }
  if (Epi::kReduce) write_partial(part, blockIdx.x, acc);
}

// Segments of the split rows in LDS slices.  The work items, slice-major (item
// i of slice x is work item x nitem + i), are dealt to the blocks in contiguous
// ranges of equal size, so that every block of the one resident wave of blocks
// gets the same share; a block stages u over each slice its range touches
// ([x LSLICE, (x+1) LSLICE) of the samples, at most a few) in LDS and takes that
// slice's items.  An item is LTB / lpr rows of one bin, lpr lanes per row; a
// lane loads LVEC offsets at a time (LXV loads in flight) and adds the LDS
// values they name.
template <typename V>
__global__ __launch_bounds__(LTB) void k_xt_lds(XtLds L, const V* __restrict__ u, State* st, int solve) {
  if (solve && st->stop) return;
  extern __shared__ double lds_raw[];
  V* lu = reinterpret_cast<V*>(lds_raw);  // LSLICE + 1 values: the slice, then the zero slot
  const int tid = threadIdx.x;
  const long long total = (long long)L.nslice * L.nitem;
  const int w0 = (int)(total * blockIdx.x / L.nblk), w1 = (int)(total * (blockIdx.x + 1) / L.nblk);
  const uint4* xv = reinterpret_cast<const uint4*>(L.xcol);
  constexpr unsigned PAD2 = (unsigned)LSLICE | ((unsigned)LSLICE << 16);  // two padding offsets
  for (int w = w0; w < w1;) {
    const int x = w / L.nitem;
    const int wend = min(w1, (x + 1) * L.nitem);
    __syncthreads();  // every wave is done with the previous slice
    const int x0 = x * LSLICE;
    const int len = min(LSLICE, L.n - x0);
    stage_lds<LTB, 8>(lu, u + x0, len);
    if (tid == 0) lu[LSLICE] = (V)0;
    __syncthreads();
    const int* xp = L.xptr + (long long)x * (L.nsplit + 1);
    for (int it = w - x * L.nitem; it < wend - x * L.nitem; it++) {
      int b = 0;
      while (it >= L.item0[b + 1]) b++;
      const int lpr = L.lpr[b];
      const int j = L.row0[b] + (it - L.item0[b]) * (LTB / lpr) + tid / lpr;
      const int lane = tid & (lpr - 1);
      const bool live = j < L.row0[b + 1];
      V v = (V)0;
      if (live) {
        const int ve = xp[j + 1] / LVEC;
        for (int k0 = xp[j] / LVEC + lane; k0 < ve; k0 += lpr * LXV) {
          uint4 q[LXV];
#pragma unroll
          for (int e = 0; e < LXV; e++) {
            const int k = k0 + e * lpr;
            q[e] = k < ve ? xv[k] : make_uint4(PAD2, PAD2, PAD2, PAD2);
          }
#pragma unroll
          for (int e = 0; e < LXV; e++) {
            const unsigned wd[4] = {q[e].x, q[e].y, q[e].z, q[e].w};
#pragma unroll
            for (int h = 0; h < 4; h++) v += lu[wd[h] & 0xffffu] + lu[wd[h] >> 16];
          }
        }
      }
      for (int o = lpr >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (live && lane == 0) L.parts[(long long)x * L.nsplit + j] = (double)v;
    }
    w = wend;
  }
}

// Slice-major copy of the split rows' indices for the LDS slices: thread (x, j)
// copies row j's segment of slice x ([segp[x nsplit + j], segp[(x+1) nsplit + j]))
// to xcol[xptr[x (nsplit+1) + j] ..] as offsets from the slice's first sample,
// then fills the rest of its entries (up to the next segment's start) with LSLICE.
__global__ __launch_bounds__(BS) void k_slice_copy(const int* __restrict__ col, const int* __restrict__ segp,
                                                   const int* __restrict__ xptr, int nsplit, int nslice,
                                                   unsigned short* xcol) {
  const long long t = (long long)blockIdx.x * BS + threadIdx.x;
  if (t >= (long long)nslice * nsplit) return;
  const int x = (int)(t / nsplit), j = (int)(t % nsplit);
  const int b = segp[(long long)x * nsplit + j], e = segp[(long long)(x + 1) * nsplit + j];
  const int o = xptr[(long long)x * (nsplit + 1) + j], o1 = xptr[(long long)x * (nsplit + 1) + j + 1];
  const int x0 = x * LSLICE;
  for (int k = b; k < e; k++) xcol[o + (k - b)] = (unsigned short)(col[k] - x0);
  for (int k = o + (e - b); k < o1; k++) xcol[k] = (unsigned short)LSLICE;
}

// Slice boundaries of the split rows of X^T: segp[x * nsplit + j] is the first
// nonzero k of row j with col[k] >= the first sample of slice x (the row's end
// if none), for x = 0..nslice.  Slice x starts at x n / nslice (slice_len 0:
// XCD slices) or at min(x slice_len, n) (LDS slices).  Sample indices increase
// along a row of X^T.
__global__ __launch_bounds__(BS) void k_slice_bounds(const int* __restrict__ rowptr, const int* __restrict__ col,
                                                     int nsplit, long long n, int nslice, int slice_len, int* segp) {
  const long long t = (long long)blockIdx.x * BS + threadIdx.x;
  if (t >= (long long)(nslice + 1) * nsplit) return;
  const int x = (int)(t / nsplit), j = (int)(t % nsplit);
  const long long start = slice_len > 0 ? (long long)x * slice_len : (long long)x * n / nslice;
  const int key = (int)(start < n ? start : n);
  int lo = rowptr[j], hi = rowptr[j + 1];
  while (lo < hi) {
    const int mid = lo + (hi - lo) / 2;
    if (col[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  segp[t] = lo;
}

// Multi-part rows r0 + [0, nlong) of an X^T product (the rows of several
// chunks, or with XCD slices every XCD-split row): row r0 + j is the ordered sum
// of its parts lpart[row_chunk0[j] .. row_chunk0[j+1]).  Partial in slot `slot`.
// In a solve (solve != 0) nothing runs once every shift has stopped.
template <class Epi>
__global__ __launch_bounds__(BS) void k_assemble(int r0, int nlong, const int* row_chunk0, const double* lpart,
                                                 Epi epi, State* st, double* part, int slot, int solve) {
  if (solve && st->stop) return;
  epi.prepare(st);
  double acc = 0.0;
  for (int j = blockIdx.x * BS + threadIdx.x; j < nlong; j += gridDim.x * BS) {
    const int c0 = row_chunk0[j], c1 = row_chunk0[j + 1];
    double v = 0.0;
    for (int k = c0; k < c1; k += 8) {
      double x[8];
#pragma unroll
      for (int e = 0; e < 8; e++) x[e] = k + e < c1 ? lpart[k + e] : 0.0;
#pragma unroll
      for (int e = 0; e < 8; e++) v += x[e];
    }
    acc += epi.row(r0 + j, (typename Epi::V)v);
  }
  if (Epi::kReduce) write_partial(part, slot + blockIdx.x, acc);
}

// ---------------------------------------------------------------------------
// streaming kernels of the recurrence
// ---------------------------------------------------------------------------

// r_0 = b (ring slot 0), p_0 = b, P_s = b, W_s = 0; partials of <b, b> (also
// the first <p, p>).  Launched with the grid of k_pupdate.
// With labw (sample-space solves), also partials of sum_j labw_j p_j into lpart.
template <typename V>
__global__ __launch_bounds__(BS) void k_init(const double* __restrict__ b, V* ring, V* p, V* P, long long ldp, double* W,
                                             long long d, int nshift, double* part, const double* labw,
                                             double* lpart) {
  double acc = 0.0, lac = 0.0;
  for (long long j = (long long)blockIdx.x * BS + threadIdx.x; j < d; j += (long long)gridDim.x * BS) {
    const V x = (V)b[j];
    ring[j] = x;
    p[j] = x;
    for (int s = 0; s < nshift; s++) {
      P[s * ldp + j] = x;
      W[s * d + j] = 0.0;
    }
    acc += (double)x * (double)x;
    if (labw) lac += labw[j] * (double)x;
  }
  write_partial(part, blockIdx.x, acc);
  if (labw) write_partial(lpart, blockIdx.x, lac);
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

// Residual update as a pass of its own (the sample-space solve): <p, q> =
// <t, u> + sigma0 <p, p> from the partials of the graph product
// and of the previous direction update; a_i = <r,r>/<p,q>; r_{i+1} = r_i - a_i q
// into the next ring slot, where q_j of a long row j < nlong is the ordered sum
// of its chunk sums plus sigma0 p_j; partials of <r_{i+1}, r_{i+1}>.  The last
// block advances zeta (or flags a breakdown).  The first pass's vector loads
// are issued before the partial sums, so both latencies overlap.
template <typename V>
__global__ __launch_bounds__(BS) void k_resid(State* st, const V* __restrict__ q, const V* __restrict__ p,
                                              V* ring, long long ldd, long long d, const double* tu_part, int ntu,
                                              const double* pp_part, int npp, int nlong,
                                              const int* __restrict__ row_chunk0, const double* __restrict__ lpart,
                                              double* part) {
  if (st->stop) return;
  const double sigma0 = st->sigma0;
  const int i = st->iter, m = st->chunk;
  const V* r = ring + (long long)(i % m) * ldd;
  V* rn = ring + (long long)((i + 1) % m) * ldd;
  const long long step = (long long)gridDim.x * BS * UNR;
  long long j0 = (long long)blockIdx.x * BS * UNR + threadIdx.x;
  double rv[UNR], qv[UNR];
  auto load = [&]() {
#pragma unroll
    for (int u = 0; u < UNR; u++) {
      const long long j = j0 + (long long)u * BS;
      rv[u] = j < d ? (double)r[j] : 0.0;
      if (j < nlong) {  // sum the row's chunk sums in order, 8 loads in flight
        const int c0 = row_chunk0[j], c1 = row_chunk0[j + 1];
        double c = 0.0;
        for (int k = c0; k < c1; k += 8) {
          double x[8];
#pragma unroll
          for (int e = 0; e < 8; e++) x[e] = k + e < c1 ? lpart[k + e] : 0.0;
#pragma unroll
          for (int e = 0; e < 8; e++) c += x[e];
        }
        qv[u] = (double)(V)c + (double)((V)sigma0 * p[j]);
      } else {
        qv[u] = j < d ? (double)q[j] : 0.0;
      }
    }
  };
  load();
  const double pq = sum_partials(tu_part, ntu) + sigma0 * sum_partials(pp_part, npp);
  const double a = st->rr / pq;
  const bool ok = (pq > 0.0) && isfinite(a);
  double acc = 0.0;
  if (ok) {
    for (;;) {
#pragma unroll
      for (int u = 0; u < UNR; u++) {
        const long long j = j0 + (long long)u * BS;
        const V x = (V)(rv[u] - a * qv[u]);
        if (j < d) rn[j] = x;
        acc += (double)x * (double)x;
      }
      j0 += step;
      if (j0 >= d) break;
      load();
    }
  }
  write_partial(part, blockIdx.x, acc);
  if (last_block(st, TK_STEP)) {
    if (ok) {
      step_scalars(st, a);
    } else if (threadIdx.x == 0) {
      st->status = FSDA_E_BREAKDOWN;
      st->stop = 1;
    }
  }
}

// r_{i+1,j} of a long row j < nlong of X^T (the fused X^T pass leaves these
// rows as chunk sums): q_j is the ordered sum of the row's chunk sums plus
// sigma0 p_j, and r_{i+1,j} = r_{i,j} - a_i q_j.  Returns r_{i+1,j} and p_j.
struct LongRow {
  double r, p;
};
template <typename V>
__device__ __forceinline__ LongRow long_row_residual(int j, const int* __restrict__ row_chunk0,
                                                     const double* __restrict__ lpart, const V* p, const V* r,
                                                     double a, double sigma0) {
  const int c0 = row_chunk0[j], c1 = row_chunk0[j + 1];
  const V pv = p[j];
  const V rv = r[j];
  double c = 0.0;
  for (int k = c0; k < c1; k += 8) {
    double x[8];
#pragma unroll
    for (int e = 0; e < 8; e++) x[e] = k + e < c1 ? lpart[k + e] : 0.0;
#pragma unroll
    for (int e = 0; e < 8; e++) c += x[e];
  }
  const double q = (double)(V)c + (double)((V)sigma0 * pv);
  return LongRow{(double)(V)((double)rv - a * q), (double)pv};
}

// Direction update: b_{i+1} = <r_{i+1},r_{i+1}>/<r_i,r_i>; p_{i+1} = r_{i+1} + b_{i+1} p_i, with
// partials of <p_{i+1}, p_{i+1}> (and, with labw, of sum_j labw_j p_j for the
// next sample-space centring).  The last block runs the per-shift scalar
// updates and the stop test.
//
// After the fused X^T pass (step != 0) this kernel also finishes the long rows
// [0, nlong).  Every block computes their r_{i+1} (same values, same order),
// for <r_{i+1}, r_{i+1}> = (partials of the X^T pass) + (long rows).  Their
// r_{i+1} and p_{i+1} are stored by the last block only, since every block
// reads r_i and p_i there (with a fold interval of 1, r_i and r_{i+1} share a
// ring slot); and the last block first advances zeta with the step a_i that
// the X^T pass published.
constexpr int LCACHE = 4;  // long rows per thread kept in registers for the last block's stores
template <typename V>
__global__ __launch_bounds__(BS) void k_pupdate(State* st, V* ring, V* p, long long ldd, long long d,
                                                const double* rr_part, int nrr, double* hist, double* pp_part,
                                                const double* labw, double* lpart, int step, int nlong,
                                                const int* __restrict__ row_chunk0,
                                                const double* __restrict__ chunk_sum) {
  if (st->stop) return;
  const int i = st->iter, m = st->chunk;
  V* r = ring + (long long)((i + 1) % m) * ldd;
  const V* rprev = ring + (long long)(i % m) * ldd;
  const double a = step ? st->a_new : 0.0;
  const bool ok = !step || (st->pq_new > 0.0 && isfinite(a));
  const double sigma0 = st->sigma0;
  ShiftRegs q{};
  if (step) q = load_shift_regs(st);
  const long long gstep = (long long)gridDim.x * BS * UNR;
  long long j0 = (long long)blockIdx.x * BS * UNR + threadIdx.x;
  double rv[UNR], pv[UNR];
  double acc = 0.0, lac = 0.0, rrn = 0.0, b = 0.0;
  double lx[LCACHE], lp[LCACHE];
  if (ok) {
    // first elements of this block, in flight during the sums below
#pragma unroll
    for (int u = 0; u < UNR; u++) {
      const long long j = j0 + (long long)u * BS;
      if (j < nlong) {
        const LongRow lr = long_row_residual<V>((int)j, row_chunk0, chunk_sum, p, rprev, a, sigma0);
        rv[u] = lr.r;
        pv[u] = lr.p;
      } else {
        rv[u] = j < d ? (double)r[j] : 0.0;
        pv[u] = j < d ? (double)p[j] : 0.0;
      }
    }
    double rl = 0.0;  // the long rows' part of <r_{i+1}, r_{i+1}>
#pragma unroll
    for (int k = 0; k < LCACHE; k++) {
      const int j = threadIdx.x + k * BS;
      lx[k] = lp[k] = 0.0;
      if (j < nlong) {
        const LongRow lr = long_row_residual<V>(j, row_chunk0, chunk_sum, p, rprev, a, sigma0);
        lx[k] = lr.r;
        lp[k] = lr.p;
        rl += lr.r * lr.r;
      }
    }
    for (int j = threadIdx.x + LCACHE * BS; j < nlong; j += BS) {
      const LongRow lr = long_row_residual<V>(j, row_chunk0, chunk_sum, p, rprev, a, sigma0);
      rl += lr.r * lr.r;
    }
    rrn = sum_partials(rr_part, nrr) + (nlong > 0 ? block_sum_all(rl) : 0.0);
    b = rrn / st->rr;
    for (;;) {
#pragma unroll
      for (int u = 0; u < UNR; u++) {
        const long long j = j0 + (long long)u * BS;
        const V x = (V)(rv[u] + b * pv[u]);
        if (j < d && j >= nlong) p[j] = x;
        acc += j < d ? (double)x * (double)x : 0.0;
        if (labw && j < d) lac += labw[j] * (double)x;
      }
      j0 += gstep;
      if (j0 >= d) break;
#pragma unroll
      for (int u = 0; u < UNR; u++) {
        const long long j = j0 + (long long)u * BS;
        if (j < nlong) {
          const LongRow lr = long_row_residual<V>((int)j, row_chunk0, chunk_sum, p, rprev, a, sigma0);
          rv[u] = lr.r;
          pv[u] = lr.p;
        } else {
          rv[u] = j < d ? (double)r[j] : 0.0;
          pv[u] = j < d ? (double)p[j] : 0.0;
        }
      }
    }
  }
  write_partial(pp_part, blockIdx.x, acc);
  if (labw) write_partial(lpart, blockIdx.x, lac);
  if (last_block(st, TK_DIR)) {
    if (!ok) {
      if (threadIdx.x == 0) {
        st->status = FSDA_E_BREAKDOWN;
        st->stop = 1;
      }
    } else {
      // r_{i+1}, p_{i+1} of the long rows: every other block has finished reading r_i, p_i
#pragma unroll
      for (int k = 0; k < LCACHE; k++) {
        const int j = threadIdx.x + k * BS;
        if (j < nlong) {
          r[j] = (V)lx[k];
          p[j] = (V)(lx[k] + b * lp[k]);
        }
      }
      for (int j = threadIdx.x + LCACHE * BS; j < nlong; j += BS) {
        const LongRow lr = long_row_residual<V>(j, row_chunk0, chunk_sum, p, rprev, a, sigma0);
        r[j] = (V)lr.r;
        p[j] = (V)(lr.r + b * lr.p);
      }
      if (step)
        step_resid_scalars(st, q, i, a, rrn, b, hist);
      else
        resid_scalars(st, rrn, b, hist);
    }
  }
}

// Fold of iterations [fold_start, iter) into the per-shift state.  Per shift s
// the iterations k = 0 .. cnt-1 of the chunk apply
//   W_s += a_k P_s ;  P_s = zeta_k r_k + b_k P_s       (Alg. 3; r_k the residual of iteration fold_start + k + 1)
// (a frozen shift carries the identity step a = zeta = 0, b = 1).  Unrolled,
//   W_s <- W_s + A_s P_s + sum_k H_k,s r_k ,   P_s <- B_s P_s + sum_k G_k,s r_k
// with, backwards from G'_{cnt-1} = 0 and E_{cnt-1} = 1,
//   H_k = zeta_k G'_k, G_k = zeta_k E_k,  G'_{k-1} = a_k + b_k G'_k,  E_{k-1} = b_k E_k,
//   A_s = G'_{-1}, B_s = E_{-1}.
// k_fold_coef (one block, one thread per shift) computes the coefficients;
// k_fold_apply streams the buffered residuals once per group of FG shifts and
// reads and writes W_s and P_s once per chunk: a (2 FG x cnt) by (cnt x d)
// contraction plus the two scalings, per chunk instead of per iteration.
constexpr int FG = 16;  // shifts per pass over the buffered residuals
struct FoldCoef {
  double h[MAXCHUNK][MAXS];  // H_k,s
  double g[MAXCHUNK][MAXS];  // G_k,s
  double a[MAXS], b[MAXS];   // A_s, B_s
  int on[MAXS];              // shift active at the first iteration of the chunk
};

__global__ __launch_bounds__(BS) void k_fold_coef(const State* st, const double* __restrict__ hist,
                                                  FoldCoef* __restrict__ cf, int nshift) {
  const int k0 = st->fold_start, cnt = st->iter - k0, m = st->chunk;
  const int s = threadIdx.x;
  if (cnt <= 0 || s >= nshift) return;
  constexpr int KB = 16;  // steps whose coefficients are loaded together
  double gp = 0.0, e = 1.0;
  for (int kb = cnt - 1; kb >= 0; kb -= KB) {
    double a[KB], z[KB], b[KB];
#pragma unroll
    for (int u = 0; u < KB; u++) {
      const int k = kb - u;
      const double* h = hist + ((size_t)((k0 + (k >= 0 ? k : 0)) % m) * MAXS + s) * 4;
      a[u] = h[0];
      z[u] = h[1];
      b[u] = h[2];
    }
#pragma unroll
    for (int u = 0; u < KB; u++) {
      const int k = kb - u;
      if (k >= 0) {
        cf->h[k][s] = z[u] * gp;
        cf->g[k][s] = z[u] * e;
        gp = a[u] + b[u] * gp;
        e = b[u] * e;
      }
    }
  }
  cf->a[s] = gp;
  cf->b[s] = e;
  cf->on[s] = hist[((size_t)(k0 % m) * MAXS + s) * 4 + 3] != 0.0;
}

template <typename V>
__global__ __launch_bounds__(BS) void k_fold_apply(const State* st, const FoldCoef* __restrict__ cf, const V* ring,
                                                   long long ldd, double* W, long long d, V* P, long long ldp,
                                                   int nshift) {
  const int k0 = st->fold_start, cnt = st->iter - k0, m = st->chunk;
  if (cnt <= 0) return;
  const int first = (k0 + 1) % m;
  constexpr int KU = 8;  // buffered residuals in flight
  for (long long j = (long long)blockIdx.x * BS + threadIdx.x; j < d; j += (long long)gridDim.x * BS) {
    for (int s0 = 0; s0 < nshift; s0 += FG) {
      double ah[FG], ag[FG];
#pragma unroll
      for (int g = 0; g < FG; g++) ah[g] = ag[g] = 0.0;
      for (int k = 0; k < cnt; k += KU) {
        double rv[KU];
#pragma unroll
        for (int u = 0; u < KU; u++) {  // slot (k0 + k + u + 1) mod m: the chunk wraps the ring at most once
          const int sl = first + k + u;
          rv[u] = k + u < cnt ? (double)ring[(long long)(sl < m ? sl : sl - m) * ldd + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < KU; u++) {
          if (k + u < cnt) {
            const double* hk = cf->h[k + u] + s0;
            const double* gk = cf->g[k + u] + s0;
#pragma unroll
            for (int g = 0; g < FG; g++) {
              ah[g] += hk[g] * rv[u];
              ag[g] += gk[g] * rv[u];
            }
          }
        }
      }
#pragma unroll
      for (int g = 0; g < FG; g++) {
        const int s = s0 + g;
        if (s < nshift && cf->on[s]) {
          const double p = (double)P[s * ldp + j];
          W[s * d + j] += cf->a[s] * p + ah[g];
          P[s * ldp + j] = (V)(cf->b[s] * p + ag[g]);  // P_s is stored in V
        }
      }
    }
  }
}

__global__ void k_fold_done(State* st) { st->fold_start = st->iter; }

// Measurement aid: per block, the sum of src[idx[k]] over a grid-stride share
// of k (UNR independent gathers in flight per thread), one partial per block.
// It isolates the rate of random 8-byte gathers, which bounds the products.
__global__ __launch_bounds__(BS) void k_gather_sum(const double* __restrict__ src, const int* __restrict__ idx,
                                                   long long nidx, double* part) {
  double acc = 0.0;
  const long long stride = (long long)gridDim.x * BS;
  for (long long k0 = (long long)blockIdx.x * BS + threadIdx.x; k0 < nidx; k0 += stride * UNR) {
    int ii[UNR];
    double g[UNR];
#pragma unroll
    for (int u = 0; u < UNR; u++) {
      const long long k = k0 + (long long)u * stride;
      ii[u] = k < nidx ? idx[k] : -1;
    }
#pragma unroll
    for (int u = 0; u < UNR; u++) g[u] = ii[u] >= 0 ? src[ii[u]] : 0.0;
#pragma unroll
    for (int u = 0; u < UNR; u++) acc += g[u];
  }
  write_partial(part, blockIdx.x, acc);
}

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
// dst[j] = f * sum(partials) * src[j]
__global__ __launch_bounds__(BS) void k_scaled_d(const double* __restrict__ src, double* dst, long long n,
                                                 const double* part, int np, double f) {
  const double c = f * sum_partials(part, np);
  FSDA_GRID_LOOP(j, n) dst[j] = c * src[j];
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



__global__ void k_expand_rows(const int* rowptr, long long nrows, int* rowid) {
  FSDA_GRID_LOOP(r, nrows) for (int k = rowptr[r]; k < rowptr[r + 1]; k++) rowid[k] = (int)r;
}

// Split the rows of X (internal column ids) into the mask features [0, mtop)
// and the rest: mask[r] gets a bit per mask feature, cnt[r] the number of others.
__global__ void k_mask_split(const int* rowptr, const int* col, long long nrows, int mtop, unsigned long long* mask,
                             int* cnt) {
  FSDA_GRID_LOOP(r, nrows) {
    unsigned long long m = 0;
    int c = 0;
    for (int k = rowptr[r]; k < rowptr[r + 1]; k++) {
      const int j = col[k];
      if (j < mtop)
        m |= 1ull << j;
      else
        c++;
    }
    mask[r] = m;
    cnt[r] = c;
  }
}

// The other features of each row, in order, at rrowptr[r].
__global__ void k_mask_fill(const int* rowptr, const int* col, long long nrows, int mtop, const int* rrowptr,
                            int* rcol) {
  FSDA_GRID_LOOP(r, nrows) {
    int o = rrowptr[r];
    for (int k = rowptr[r]; k < rowptr[r + 1]; k++) {
      const int j = col[k];
      if (j >= mtop) rcol[o++] = j;
    }
  }
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
