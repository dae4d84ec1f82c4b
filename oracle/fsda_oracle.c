/*
 * CPU oracle for fast semi-supervised discriminant analysis (FSDA) -- TEST
 * INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use this file; the GPU library neither links nor calls it.
 *
 * Plain FP64, written from the paper's statement of the problem:
 *
 *   For every regularisation value beta > 0, solve (Alg. 7, step 4)
 *       ( Xc^T [ (1-alpha) P_l + alpha L ] X + beta I_D ) w = Xc^T [W 0; 0 0] X r
 *   with Xc = X - 1 mu_l^T the data centred on the labeled mean (Sec. 3.2.3),
 *   mu_l = X^T 1_l / l, P_l the labeled-row selector and L = D - S the
 *   unnormalised graph Laplacian (Sec. 2.3).  W is the labeled between-class
 *   weight: W_ij = 1/N_c when rows i and j are both labeled with class c
 *   (Sec. 2.1).
 *
 * Readings (the paper leaves these open):
 *   - the operator is applied two-sided, Xc^T M Xc, with both centred products
 *     of Sec. 3.2.3 written out; the paper notes one centred product suffices,
 *     so the result equals the one-sided Xc^T M X of Alg. 7;
 *   - the canonical right-hand side is b = Xc^T y_c, y_c = labels minus their
 *     labeled mean (0 on unlabeled rows); for two classes the Alg. 7 right-hand
 *     side is a scalar multiple of it, the scalar depending on the random r.
 *     orc_rhs() computes either form;
 *   - CG (Alg. 2) runs to ||r|| <= rtol ||b|| (relative instead of absolute);
 *   - each shift is solved by its own CG: no shift recurrence here at all.
 *
 * Reductions use fixed chunks summed in a fixed order, so results do not depend
 * on the OpenMP thread count.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC fsda_oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int64_t n, d;
  const int32_t *x_rowptr, *x_col; /* X: n x d binary, CSR without values */
  const int32_t *s_rowptr, *s_col; /* S: n x n binary symmetric similarity */
  int64_t n_lab;
  const int32_t *lab_idx; /* labeled rows */
  const int8_t *lab_y;    /* their labels, +1 / -1 */
  double alpha;           /* weight of the manifold term, 0 <= alpha <= 1 */
} orc_problem;

/* Derived data: labeled mask, degrees, mu_l and the transpose of X. */
typedef struct {
  const orc_problem *pb;
  uint8_t *lab;     /* [n] 1 if labeled */
  double *ycen;     /* [n] centred labels, 0 on unlabeled rows */
  double *deg;      /* [n] d_i = sum_j s_ij */
  double *mu;       /* [d] labeled mean sample */
  int64_t *t_rowptr;/* [d+1] transpose of X (rows = features) */
  int32_t *t_col;   /* [nnz] sample ids */
  double *v, *t;    /* [n] scratch */
} orc_ctx;

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_E_ARG = -1, ORC_E_LABELS = -3, ORC_E_BREAKDOWN = -5 };

#define NCHUNK 256

/* ---- reductions in a fixed order ---------------------------------------- */
static double dot(int64_t m, const double *a, const double *b) {
  double part[NCHUNK];
#pragma omp parallel for schedule(static)
  for (int c = 0; c < NCHUNK; c++) {
    int64_t lo = m * c / NCHUNK, hi = m * (c + 1) / NCHUNK;
    double s = 0.0;
    for (int64_t i = lo; i < hi; i++) s += a[i] * b[i];
    part[c] = s;
  }
  double s = 0.0;
  for (int c = 0; c < NCHUNK; c++) s += part[c];
  return s;
}
static double total(int64_t m, const double *a) {
  double part[NCHUNK];
#pragma omp parallel for schedule(static)
  for (int c = 0; c < NCHUNK; c++) {
    int64_t lo = m * c / NCHUNK, hi = m * (c + 1) / NCHUNK;
    double s = 0.0;
    for (int64_t i = lo; i < hi; i++) s += a[i];
    part[c] = s;
  }
  double s = 0.0;
  for (int c = 0; c < NCHUNK; c++) s += part[c];
  return s;
}

/* ---- plain sparse products ---------------------------------------------- */
/* out = X v : out_i = sum of v_j over the features j of sample i */
static void x_mul(const orc_problem *pb, const double *v, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < pb->n; i++) {
    double s = 0.0;
    for (int32_t k = pb->x_rowptr[i]; k < pb->x_rowptr[i + 1]; k++) s += v[pb->x_col[k]];
    out[i] = s;
  }
}
/* out = X^T u : out_j = sum of u_i over the samples i that have feature j */
static void xt_mul(const orc_ctx *c, const double *u, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < c->pb->d; j++) {
    double s = 0.0;
    for (int64_t k = c->t_rowptr[j]; k < c->t_rowptr[j + 1]; k++) s += u[c->t_col[k]];
    out[j] = s;
  }
}

/* ---- centred products of Sec. 3.2.3 -------------------------------------- */
/* (X - 1 mu^T) v = X v - 1 <mu, v> */
static void xc_mul(const orc_ctx *c, const double *v, double *out) {
  const orc_problem *pb = c->pb;
  x_mul(pb, v, out);
  double m = dot(pb->d, c->mu, v);
  for (int64_t i = 0; i < pb->n; i++) out[i] -= m;
}
/* (X - 1 mu^T)^T u = X^T u - mu <1, u> */
static void xct_mul(const orc_ctx *c, const double *u, double *out) {
  const orc_problem *pb = c->pb;
  xt_mul(c, u, out);
  double s = total(pb->n, u);
  for (int64_t j = 0; j < pb->d; j++) out[j] -= c->mu[j] * s;
}

/* M t = (1-alpha) P_l t + alpha (D - S) t   (Eq. SDAeig, Sec. 2.3) */
static void m_mul(const orc_ctx *c, const double *t, double *out) {
  const orc_problem *pb = c->pb;
  double a = pb->alpha;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < pb->n; i++) {
    double st = 0.0;
    for (int32_t k = pb->s_rowptr[i]; k < pb->s_rowptr[i + 1]; k++) st += t[pb->s_col[k]];
    double lt = c->deg[i] * t[i] - st;
    out[i] = (1.0 - a) * (c->lab[i] ? t[i] : 0.0) + a * lt;
  }
}

/* ---- context ------------------------------------------------------------- */
static void ctx_free(orc_ctx *c) {
  free(c->lab); free(c->ycen); free(c->deg); free(c->mu);
  free(c->t_rowptr); free(c->t_col); free(c->v); free(c->t);
  memset(c, 0, sizeof(*c));
}

static int ctx_init(orc_ctx *c, const orc_problem *pb) {
  memset(c, 0, sizeof(*c));
  c->pb = pb;
  int64_t n = pb->n, d = pb->d, nnz = pb->x_rowptr[n];
  if (n <= 0 || d <= 0 || pb->n_lab < 2) return ORC_E_ARG;
  c->lab = (uint8_t *)calloc((size_t)n, 1);
  c->ycen = (double *)calloc((size_t)n, sizeof(double));
  c->deg = (double *)calloc((size_t)n, sizeof(double));
  c->mu = (double *)calloc((size_t)d, sizeof(double));
  c->t_rowptr = (int64_t *)calloc((size_t)d + 1, sizeof(int64_t));
  c->t_col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  c->v = (double *)malloc(sizeof(double) * (size_t)n);
  c->t = (double *)malloc(sizeof(double) * (size_t)n);
  /* labels: y_c = y - mean over labeled rows of y */
  int64_t npos = 0, nneg = 0;
  double ysum = 0.0;
  for (int64_t k = 0; k < pb->n_lab; k++) {
    int32_t i = pb->lab_idx[k];
    if (i < 0 || i >= n || c->lab[i]) { ctx_free(c); return ORC_E_ARG; }
    c->lab[i] = 1;
    if (pb->lab_y[k] > 0) npos++; else nneg++;
    ysum += pb->lab_y[k] > 0 ? 1.0 : -1.0;
  }
  if (npos == 0 || nneg == 0) { ctx_free(c); return ORC_E_LABELS; }
  double ybar = ysum / (double)pb->n_lab;
  for (int64_t k = 0; k < pb->n_lab; k++)
    c->ycen[pb->lab_idx[k]] = (pb->lab_y[k] > 0 ? 1.0 : -1.0) - ybar;
  /* degrees d_i = number of neighbours */
  for (int64_t i = 0; i < n; i++) c->deg[i] = (double)(pb->s_rowptr[i + 1] - pb->s_rowptr[i]);
  /* transpose of X by counting */
  for (int64_t k = 0; k < nnz; k++) c->t_rowptr[pb->x_col[k] + 1]++;
  for (int64_t j = 0; j < d; j++) c->t_rowptr[j + 1] += c->t_rowptr[j];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)d);
  memcpy(fill, c->t_rowptr, sizeof(int64_t) * (size_t)d);
  for (int64_t i = 0; i < n; i++)
    for (int32_t k = pb->x_rowptr[i]; k < pb->x_rowptr[i + 1]; k++) c->t_col[fill[pb->x_col[k]]++] = (int32_t)i;
  free(fill);
  /* l mu_l = X^T 1_l  (Alg. 7, step 3) */
  for (int64_t i = 0; i < n; i++) c->v[i] = c->lab[i] ? 1.0 : 0.0;
  xt_mul(c, c->v, c->mu);
  for (int64_t j = 0; j < d; j++) c->mu[j] /= (double)pb->n_lab;
  return ORC_OK;
}

/* q = (Xc^T M Xc + beta I) p */
static void apply_ctx(orc_ctx *c, double beta, const double *p, double *q) {
  xc_mul(c, p, c->v);
  m_mul(c, c->v, c->t);
  xct_mul(c, c->t, q);
  for (int64_t j = 0; j < c->pb->d; j++) q[j] += beta * p[j];
}

/* ---- public entry points -------------------------------------------------- */
void orc_set_threads(int nt) {
#ifdef _OPENMP
  if (nt > 0) omp_set_num_threads(nt);
#else
  (void)nt;
#endif
}
int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* mu_l = X^T 1_l / l */
int orc_mean_labeled(const orc_problem *pb, double *mu) {
  orc_ctx c;
  int rc = ctx_init(&c, pb);
  if (rc) return rc;
  memcpy(mu, c.mu, sizeof(double) * (size_t)pb->d);
  ctx_free(&c);
  return ORC_OK;
}

/* q = (Xc^T M Xc + beta I) p for one vector */
int orc_apply(const orc_problem *pb, double beta, const double *p, double *q) {
  orc_ctx c;
  int rc = ctx_init(&c, pb);
  if (rc) return rc;
  apply_ctx(&c, beta, p, q);
  ctx_free(&c);
  return ORC_OK;
}

/* u = M t in sample space (exposed for the annihilation check of Sec. 3.2.3) */
int orc_m_apply(const orc_problem *pb, const double *t, double *u) {
  orc_ctx c;
  int rc = ctx_init(&c, pb);
  if (rc) return rc;
  m_mul(&c, t, u);
  ctx_free(&c);
  return ORC_OK;
}

/* u = Xc^T v for an arbitrary sample-space vector v */
int orc_xct(const orc_problem *pb, const double *v, double *u) {
  orc_ctx c;
  int rc = ctx_init(&c, pb);
  if (rc) return rc;
  xct_mul(&c, v, u);
  ctx_free(&c);
  return ORC_OK;
}

/* Right-hand side.
 * r == NULL : b = Xc^T y_c (canonical);
 * r != NULL : b = Xc^T [W 0; 0 0] X r (Alg. 7, step 4), W_ij = 1/N_c on the
 *             class blocks of the labeled rows. */
int orc_rhs(const orc_problem *pb, const double *r, double *b) {
  orc_ctx c;
  int rc = ctx_init(&c, pb);
  if (rc) return rc;
  int64_t n = pb->n;
  if (r == NULL) {
    xct_mul(&c, c.ycen, b);
  } else {
    x_mul(pb, r, c.t);
    double sp = 0.0, sn = 0.0;
    int64_t np = 0, nn = 0;
    for (int64_t k = 0; k < pb->n_lab; k++) {
      int32_t i = pb->lab_idx[k];
      if (pb->lab_y[k] > 0) { sp += c.t[i]; np++; } else { sn += c.t[i]; nn++; }
    }
    /* ([W 0;0 0] X r)_i = (1/N_c) sum over class c of (X r), for labeled i of class c */
    for (int64_t i = 0; i < n; i++) c.v[i] = 0.0;
    for (int64_t k = 0; k < pb->n_lab; k++) {
      int32_t i = pb->lab_idx[k];
      c.v[i] = pb->lab_y[k] > 0 ? sp / (double)np : sn / (double)nn;
    }
    xct_mul(&c, c.v, b);
  }
  ctx_free(&c);
  return ORC_OK;
}

/* q = (Cl^T M + beta I_N) z in sample space, Cl = I_N - 1 1_l^T / l, applied as
 * printed in Alg. sasda (step 4): Cl^T v = v - 1_l <1, v> / l. */
static void sa_apply_ctx(orc_ctx *c, double beta, const double *z, double *q) {
  const orc_problem *pb = c->pb;
  m_mul(c, z, c->t);
  double s = total(pb->n, c->t) / (double)pb->n_lab;
  for (int64_t i = 0; i < pb->n; i++) q[i] = c->t[i] - (c->lab[i] ? s : 0.0) + beta * z[i];
}

typedef void (*apply_fn)(orc_ctx *, double, const double *, double *);

/* Conjugate gradient (Alg. 2) on A(beta) w = b, w0 = 0, A = apply, vectors of length d.
 * Alg. 2 writes gamma = -<r,r>/<p,q>, w <- w - gamma p, r <- r + gamma q. */
static int cg_ctx(orc_ctx *c, apply_fn apply, int64_t d, double beta, const double *b, double rtol, int maxit,
                  double *w, double *r, double *p, double *q, int *iters_out, double *relres_out, double *rec) {
  double bnorm = sqrt(dot(d, b, b));
  for (int64_t j = 0; j < d; j++) { w[j] = 0.0; r[j] = b[j]; p[j] = b[j]; }
  double rr = dot(d, r, r);
  double tol = rtol * bnorm;
  int it = 0, status = ORC_NOT_CONVERGED;
  if (bnorm == 0.0) status = ORC_OK;
  while (status == ORC_NOT_CONVERGED && it < maxit) {
    apply(c, beta, p, q);
    double pq = dot(d, p, q);
    if (!(pq > 0.0) || !isfinite(pq)) { status = ORC_E_BREAKDOWN; break; }
    double gamma = -rr / pq;
    if (rec) { rec[2 * it] = -gamma; rec[2 * it + 1] = 0.0; } /* step length of iteration it */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < d; j++) {
      w[j] -= gamma * p[j];
      r[j] += gamma * q[j];
    }
    it++;
    double rr_new = dot(d, r, r);
    if (sqrt(rr_new) <= tol) { status = ORC_OK; break; }
    double a = rr_new / rr;
    if (rec) rec[2 * it - 1] = a; /* direction coefficient after iteration it - 1 */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < d; j++) p[j] = r[j] + a * p[j];
    rr = rr_new;
  }
  /* true residual b - A w */
  apply(c, beta, w, q);
  for (int64_t j = 0; j < d; j++) r[j] = b[j] - q[j];
  *relres_out = bnorm > 0.0 ? sqrt(dot(d, r, r)) / bnorm : 0.0;
  *iters_out = it;
  return status;
}

/* Solve every shift independently.  b: [d] (NULL = canonical Xc^T y_c).
 * W: [nshift][d].  rec: NULL, or [nshift][2 maxit] receiving per iteration i the
 * CG step length a_i = <r,r>/<p,A p> at 2i and the direction coefficient
 * b_i = <r_{i+1},r_{i+1}>/<r_i,r_i> at 2i+1 (0 after the last iteration): the
 * Lanczos coefficients of the run (Sec. 3.2.1).
 * Returns the worst status (breakdown < 0 < not converged). */
int orc_solve(const orc_problem *pb, const double *b, int nshift, const double *betas, double rtol, int maxit,
              double *W, int *iters, double *relres, double *rec) {
  orc_ctx c;
  int rc = ctx_init(&c, pb);
  if (rc) return rc;
  int64_t d = pb->d;
  double *bb = (double *)malloc(sizeof(double) * (size_t)d);
  if (b) memcpy(bb, b, sizeof(double) * (size_t)d);
  else xct_mul(&c, c.ycen, bb);
  double *r = (double *)malloc(sizeof(double) * (size_t)d);
  double *p = (double *)malloc(sizeof(double) * (size_t)d);
  double *q = (double *)malloc(sizeof(double) * (size_t)d);
  int worst = ORC_OK;
  for (int s = 0; s < nshift; s++) {
    if (!(betas[s] > 0.0)) { worst = ORC_E_ARG; break; }
    int st = cg_ctx(&c, apply_ctx, d, betas[s], bb, rtol, maxit, W + (int64_t)s * d, r, p, q, iters + s, relres + s,
                    rec ? rec + (int64_t)s * 2 * maxit : NULL);
    if (st < 0) { worst = st; break; }
    if (st > worst) worst = st;
  }
  free(bb); free(r); free(p); free(q);
  ctx_free(&c);
  return worst;
}

/* Rating s = X w for each shift (Alg. 7, return value; uncentred). S: [nshift][n] */
int orc_project(const orc_problem *pb, const double *W, int nshift, double *S) {
  for (int s = 0; s < nshift; s++) x_mul(pb, W + (int64_t)s * pb->d, S + (int64_t)s * pb->n);
  return ORC_OK;
}

/* ---- spectral analysis for SDA (Alg. sasda) -------------------------------- */

/* Right-hand side of Alg. sasda in sample space.
 * r == NULL : g = y_c (canonical; the printed right-hand side is a multiple of it);
 * r != NULL : r' = r - 1 <1_l, r> / l (step 3), g = [W 0; 0 0] r' (step 4): on a
 *             labeled row of class c the mean of r' over the labeled rows of class c. */
int orc_sa_rhs(const orc_problem *pb, const double *r, double *g) {
  orc_ctx c;
  int rc = ctx_init(&c, pb);
  if (rc) return rc;
  int64_t n = pb->n;
  if (r == NULL) {
    memcpy(g, c.ycen, sizeof(double) * (size_t)n);
  } else {
    double sl = 0.0;
    for (int64_t k = 0; k < pb->n_lab; k++) sl += r[pb->lab_idx[k]];
    for (int64_t i = 0; i < n; i++) c.v[i] = r[i] - sl / (double)pb->n_lab;
    double sp = 0.0, sn = 0.0;
    int64_t np = 0, nn = 0;
    for (int64_t k = 0; k < pb->n_lab; k++) {
      int32_t i = pb->lab_idx[k];
      if (pb->lab_y[k] > 0) { sp += c.v[i]; np++; } else { sn += c.v[i]; nn++; }
    }
    for (int64_t i = 0; i < n; i++) g[i] = 0.0;
    for (int64_t k = 0; k < pb->n_lab; k++) {
      int32_t i = pb->lab_idx[k];
      g[i] = pb->lab_y[k] > 0 ? sp / (double)np : sn / (double)nn;
    }
  }
  ctx_free(&c);
  return ORC_OK;
}

/* q = (Cl^T M + beta I_N) z for one sample-space vector */
int orc_sa_apply(const orc_problem *pb, double beta, const double *z, double *q) {
  orc_ctx c;
  int rc = ctx_init(&c, pb);
  if (rc) return rc;
  sa_apply_ctx(&c, beta, z, q);
  ctx_free(&c);
  return ORC_OK;
}

/* Alg. sasda: every shift solved by its own CG in sample space; the ratings are
 * s = z.  g: [n] (NULL = canonical y_c).  Z: [nshift][n]. */
int orc_sa_solve(const orc_problem *pb, const double *g, int nshift, const double *betas, double rtol, int maxit,
                 double *Z, int *iters, double *relres) {
  orc_ctx c;
  int rc = ctx_init(&c, pb);
  if (rc) return rc;
  int64_t n = pb->n;
  double *gg = (double *)malloc(sizeof(double) * (size_t)n);
  if (g) memcpy(gg, g, sizeof(double) * (size_t)n);
  else memcpy(gg, c.ycen, sizeof(double) * (size_t)n);
  double *r = (double *)malloc(sizeof(double) * (size_t)n);
  double *p = (double *)malloc(sizeof(double) * (size_t)n);
  double *q = (double *)malloc(sizeof(double) * (size_t)n);
  int worst = ORC_OK;
  for (int s = 0; s < nshift; s++) {
    if (!(betas[s] > 0.0)) { worst = ORC_E_ARG; break; }
    int st = cg_ctx(&c, sa_apply_ctx, n, betas[s], gg, rtol, maxit, Z + (int64_t)s * n, r, p, q, iters + s,
                    relres + s, NULL);
    if (st < 0) { worst = st; break; }
    if (st > worst) worst = st;
  }
  free(gg); free(r); free(p); free(q);
  ctx_free(&c);
  return worst;
}

/* ---- regression phase of the spectral-regression variants ----------------- */

/* q = (X^T X + beta I_D) p: the regularised least-squares operator of the
 * regression step (Alg. optimizedSR, step 5), no graph and no centring. */
static void reg_apply_ctx(orc_ctx *c, double beta, const double *p, double *q) {
  x_mul(c->pb, p, c->v);
  xt_mul(c, c->v, q);
  for (int64_t j = 0; j < c->pb->d; j++) q[j] += beta * p[j];
}

/* (X^T X + beta I) w = X^T z for every beta, one CG per shift.  z: [n] sample
 * space; W: [nshift][d]. */
int orc_reg_solve(const orc_problem *pb, const double *z, int nshift, const double *betas, double rtol, int maxit,
                  double *W, int *iters, double *relres) {
  orc_ctx c;
  int rc = ctx_init(&c, pb);
  if (rc) return rc;
  int64_t d = pb->d;
  double *b = (double *)malloc(sizeof(double) * (size_t)d);
  xt_mul(&c, z, b);
  double *r = (double *)malloc(sizeof(double) * (size_t)d);
  double *p = (double *)malloc(sizeof(double) * (size_t)d);
  double *q = (double *)malloc(sizeof(double) * (size_t)d);
  int worst = ORC_OK;
  for (int s = 0; s < nshift; s++) {
    if (!(betas[s] > 0.0)) { worst = ORC_E_ARG; break; }
    int st = cg_ctx(&c, reg_apply_ctx, d, betas[s], b, rtol, maxit, W + (int64_t)s * d, r, p, q, iters + s,
                    relres + s, NULL);
    if (st < 0) { worst = st; break; }
    if (st > worst) worst = st;
  }
  free(b); free(r); free(p); free(q);
  ctx_free(&c);
  return worst;
}
