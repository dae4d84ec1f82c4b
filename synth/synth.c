/*
 * Seeded synthetic inputs for the semi-supervised discriminant analysis solve:
 * sparse binary "fingerprint" matrices and binary similarity graphs.
 *
 * This file generates inputs only.  It holds none of the solver's arithmetic
 * (no centring, no Laplacian, no Krylov step); both the CPU oracle and the GPU
 * path receive the arrays it writes.
 *
 * Random numbers: every draw is a pure function of (seed, stream, counter)
 * through SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014), so results do not depend on the thread count.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC synth.c -o libsynth.so
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

typedef struct { uint64_t key, ctr; } rng_t;

static inline rng_t rng_make(uint64_t seed, uint64_t stream, uint64_t item) {
  rng_t r;
  r.key = mix64(mix64(seed ^ 0x5851f42d4c957f2dULL) ^ mix64(stream * 0x2545f4914f6cdd1dULL + 1)) ^
          mix64(item + 0x632be59bd9b4e019ULL);
  r.ctr = 0;
  return r;
}
static inline uint64_t rng_u64(rng_t *r) { return mix64(r->key + (r->ctr++) * 0x9e3779b97f4a7c15ULL); }
/* uniform in [0, 1) with 53 random bits */
static inline double rng_unif(rng_t *r) { return (double)(rng_u64(r) >> 11) * (1.0 / 9007199254740992.0); }

/* Poisson(mean) by sequential inversion of the CDF. */
static int rng_poisson(rng_t *r, double mean) {
  double u = rng_unif(r), p = exp(-mean), c = p;
  int k = 0;
  while (u > c && k < 100000) {
    k++;
    p *= mean / k;
    c += p;
    if (p < 1e-300 && (double)k > mean) break;
  }
  return k;
}

/* ---------------------------------------------------------------------------
 * Fingerprint matrix X (binary, index-only CSR, sorted distinct columns).
 * Row i holds max(1, Poisson(mean_nnz)) distinct features (capped at d).
 * Features are drawn one at a time with probability proportional to
 * 1/rank^zipf_s, repeats discarded, which is exactly weighted sampling without
 * replacement.  Rank r maps to feature id perm[r] (a seeded random
 * permutation), so popular features are spread over the id range ("hashed").
 * ------------------------------------------------------------------------- */

/* pass 1: row lengths -> rowptr[n+1] (int64 to be safe; caller narrows). */
void synth_fp_rowlen(int64_t n, int64_t d, double mean_nnz, uint64_t seed, int64_t *rowptr) {
  rowptr[0] = 0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    rng_t r = rng_make(seed, 1, (uint64_t)i);
    int64_t k = rng_poisson(&r, mean_nnz);
    if (k < 1) k = 1;
    if (k > d) k = d;
    rowptr[i + 1] = k;
  }
  for (int64_t i = 0; i < n; i++) rowptr[i + 1] += rowptr[i];
}

/* seeded permutation of 0..d-1 (Fisher-Yates with the counter RNG) */
void synth_permutation(int64_t d, uint64_t seed, uint64_t stream, int32_t *perm) {
  for (int64_t i = 0; i < d; i++) perm[i] = (int32_t)i;
  rng_t r = rng_make(seed, stream, 0);
  for (int64_t i = d - 1; i > 0; i--) {
    int64_t j = (int64_t)(rng_unif(&r) * (double)(i + 1));
    if (j > i) j = i;
    int32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* pass 2: fill the columns.  cdf[d] is the normalised cumulative Zipf weight
 * over ranks (cdf[d-1] == 1), perm[d] maps rank -> feature id. */
void synth_fp_fill(int64_t n, int64_t d, const int64_t *rowptr, const double *cdf, const int32_t *perm,
                   uint64_t seed, int32_t *col) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; i++) {
    rng_t r = rng_make(seed, 2, (uint64_t)i);
    int64_t beg = rowptr[i], k = rowptr[i + 1] - rowptr[i], have = 0;
    int32_t *out = col + beg;
    int64_t guard = 0;
    while (have < k) {
      double u = rng_unif(&r);
      /* smallest rank with cdf[rank] > u */
      int64_t lo = 0, hi = d - 1;
      while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (cdf[mid] > u) hi = mid; else lo = mid + 1;
      }
      int32_t f = perm[lo];
      int dup = 0;
      for (int64_t t = 0; t < have; t++)
        if (out[t] == f) { dup = 1; break; }
      if (!dup) out[have++] = f;
      /* a very long run of repeats only happens when k is close to d */
      if (++guard > 64 * (k + 16)) {
        for (int64_t g = 0; g < d && have < k; g++) {
          int32_t ff = perm[g];
          int dd = 0;
          for (int64_t t = 0; t < have; t++)
            if (out[t] == ff) { dd = 1; break; }
          if (!dd) out[have++] = ff;
        }
      }
    }
    qsort(out, (size_t)k, sizeof(int32_t), cmp_i32);
  }
}

/* ---------------------------------------------------------------------------
 * Tanimoto k-nearest-neighbour graph.
 * Similarity T(a,b) = |a & b| / |a | b| on the binary rows.  Row i is linked
 * to every other row whose similarity is at least the k-th largest similarity
 * of row i ("ties included"), or to exactly k rows (similarity descending,
 * index ascending) when ties == 0.  The directed lists are written here; the
 * caller takes the union with the transpose (undirected edges).
 * ------------------------------------------------------------------------- */

static inline int32_t isect(const int32_t *a, int64_t na, const int32_t *b, int64_t nb) {
  int64_t i = 0, j = 0;
  int32_t c = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j]) i++;
    else if (a[i] > b[j]) j++;
    else { c++; i++; j++; }
  }
  return c;
}

typedef struct { double sim; int32_t j; } cand_t;

static int cmp_cand(const void *pa, const void *pb) {
  const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
  if (a->sim > b->sim) return -1;
  if (a->sim < b->sim) return 1;
  return (a->j > b->j) - (a->j < b->j);
}

/* Select from cand[0..nc) (unique j, j != i): write kept ids to out (capacity
 * cap), return count.  Identical similarities compare exactly because both
 * come from the same integer ratio computed the same way. */
static int64_t select_knn(cand_t *cand, int64_t nc, int k, int ties, int32_t *out, int64_t cap) {
  qsort(cand, (size_t)nc, sizeof(cand_t), cmp_cand);
  if (nc == 0) return 0;
  int64_t keep = nc < k ? nc : k;
  if (ties && keep > 0) {
    double kth = cand[keep - 1].sim;
    while (keep < nc && cand[keep].sim == kth) keep++;
  }
  if (keep > cap) keep = cap;
  for (int64_t t = 0; t < keep; t++) out[t] = cand[t].j;
  return keep;
}

static inline double tanimoto(const int32_t *a, int64_t na, const int32_t *b, int64_t nb) {
  int32_t c = isect(a, na, b, nb);
  int64_t un = na + nb - c;
  return un > 0 ? (double)c / (double)un : 0.0;
}

/* Exact kNN over all pairs, O(n^2 * nnz/row).  nbr is [n][cap], cnt[n]. */
void synth_knn_exact(int64_t n, const int64_t *rowptr, const int32_t *col, int k, int ties, int64_t cap,
                     int32_t *nbr, int64_t *cnt) {
#pragma omp parallel
  {
    cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * (size_t)(n > 1 ? n : 1));
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
      const int32_t *a = col + rowptr[i];
      int64_t na = rowptr[i + 1] - rowptr[i], nc = 0;
      for (int64_t j = 0; j < n; j++) {
        if (j == i) continue;
        cand[nc].sim = tanimoto(a, na, col + rowptr[j], rowptr[j + 1] - rowptr[j]);
        cand[nc].j = (int32_t)j;
        nc++;
      }
      cnt[i] = select_knn(cand, nc, k, ties, nbr + i * cap, cap);
    }
    free(cand);
  }
}

/* Approximate kNN: candidates from MinHash locality-sensitive hashing
 * (Broder 1997; banding as in Leskovec, Rajaraman, Ullman, "Mining of Massive
 * Datasets", ch. 3), re-ranked by the exact Tanimoto similarity.  For each of
 * `bands` bands of `rows_per_band` min-hashes the rows are sorted by band key;
 * the `window` rows on each side in that order become candidates. */
typedef struct { uint64_t key; int32_t row; } bkey_t;
static int cmp_bkey(const void *pa, const void *pb) {
  const bkey_t *a = (const bkey_t *)pa, *b = (const bkey_t *)pb;
  if (a->key < b->key) return -1;
  if (a->key > b->key) return 1;
  return (a->row > b->row) - (a->row < b->row);
}
static int cmp_i32u(const void *a, const void *b) { return cmp_i32(a, b); }

void synth_knn_lsh(int64_t n, const int64_t *rowptr, const int32_t *col, int k, int ties, int bands,
                   int rows_per_band, int window, uint64_t seed, int64_t cap, int32_t *nbr, int64_t *cnt) {
  int nh = bands * rows_per_band;
  uint64_t *mh = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n * (size_t)nh);
  uint64_t *hk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nh);
  for (int h = 0; h < nh; h++) hk[h] = mix64(seed * 1000003ULL + (uint64_t)h * 7919ULL + 17ULL);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    for (int h = 0; h < nh; h++) {
      uint64_t m = UINT64_MAX;
      for (int64_t t = rowptr[i]; t < rowptr[i + 1]; t++) {
        uint64_t v = mix64(((uint64_t)(uint32_t)col[t]) ^ hk[h]);
        if (v < m) m = v;
      }
      mh[i * nh + h] = m;
    }
  }
  /* position of each row in each band's sorted order */
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)bands);
  int32_t *where = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)bands);
#pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < bands; b++) {
    bkey_t *keys = (bkey_t *)malloc(sizeof(bkey_t) * (size_t)n);
    for (int64_t i = 0; i < n; i++) {
      uint64_t key = 0x12345678ULL + (uint64_t)b;
      for (int r = 0; r < rows_per_band; r++) key = mix64(key ^ mh[i * nh + b * rows_per_band + r]);
      keys[i].key = key;
      keys[i].row = (int32_t)i;
    }
    qsort(keys, (size_t)n, sizeof(bkey_t), cmp_bkey);
    for (int64_t p = 0; p < n; p++) {
      order[(int64_t)b * n + p] = keys[p].row;
      where[(int64_t)b * n + keys[p].row] = (int32_t)p;
    }
    free(keys);
  }
  free(mh);
  free(hk);
  int64_t maxc = (int64_t)bands * 2 * window;
#pragma omp parallel
  {
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxc + 1));
    cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * (size_t)(maxc + 1));
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
      int64_t m = 0;
      for (int b = 0; b < bands; b++) {
        int64_t p = where[(int64_t)b * n + i];
        for (int64_t q = p - window; q <= p + window; q++) {
          if (q < 0 || q >= n || q == p) continue;
          ids[m++] = order[(int64_t)b * n + q];
        }
      }
      qsort(ids, (size_t)m, sizeof(int32_t), cmp_i32u);
      const int32_t *a = col + rowptr[i];
      int64_t na = rowptr[i + 1] - rowptr[i], nc = 0;
      for (int64_t t = 0; t < m; t++) {
        if (t > 0 && ids[t] == ids[t - 1]) continue;
        int32_t j = ids[t];
        if (j == i) continue;
        cand[nc].sim = tanimoto(a, na, col + rowptr[j], rowptr[j + 1] - rowptr[j]);
        cand[nc].j = j;
        nc++;
      }
      cnt[i] = select_knn(cand, nc, k, ties, nbr + i * cap, cap);
    }
    free(ids);
    free(cand);
  }
  free(order);
  free(where);
}

/* Standard-normal draws (Box-Muller) and uniform draws, counter based. */
void synth_normal(int64_t n, uint64_t seed, uint64_t stream, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    rng_t r = rng_make(seed, stream, (uint64_t)i);
    double u1 = rng_unif(&r), u2 = rng_unif(&r);
    if (u1 < 1e-300) u1 = 1e-300;
    out[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}
void synth_uniform(int64_t n, double lo, double hi, uint64_t seed, uint64_t stream, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    rng_t r = rng_make(seed, stream, (uint64_t)i);
    out[i] = lo + (hi - lo) * rng_unif(&r);
  }
}
