/*
 * Plain FP64 CPU oracle for GADI-IR.  TEST INFRASTRUCTURE ONLY: it is linked
 * by the test-suite, the smoke check and the CPU-baseline leg of the benchmark,
 * never by the product library, and it shares no code with the GPU path.
 *
 * What it computes (all in IEEE double, no FMA contraction, row-ordered sums):
 *   - the HSS splitting H = (A + A^T)/2, S = (A - A^T)/2 of the paper's
 *     Section 4.1 equation, on the union pattern of A and A^T;
 *   - GADI-IR, Algorithm 1 of Section 2.1, with every step in double:
 *       r_k = b - A x_k                       (step 1)
 *       (alpha I + H) z_k = r_k   by CG       (step 2)
 *       (alpha I + S) y_k = (2-omega) alpha z_k by CGNE  (step 3)
 *       x_{k+1} = x_k + y_k                   (step 4)
 *     which with exact inner solves is the stationary GADI iteration of the
 *     Section 2.1 equation (the correction form).  Stop when
 *     ||r_k||_2 <= tol ||r_0||_2 (the RES of Section 4.1), x_0 as given.
 *   - Gershgorin row bounds of H and S (predictor features).
 *
 * Readings where the paper is silent: the inner tolerance is relative to the
 * current inner right-hand side; CGNE solves (alpha^2 I - S^2) w = g and sets
 * y = (alpha I - S) w, so (alpha I + S) y = g; zero inner initial guesses.
 *
 * Dot products use a fixed partition into ORACLE_CHUNKS chunks summed in
 * order, so results do not depend on the OpenMP thread count.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_CHUNKS 64

/* ORACLE_PLANT selects a deliberately wrong variant, compiled only by the
 * test that checks the pins catch it: 1 flips the sign in y = (alpha I - S) w,
 * 2 uses (1 - omega) alpha for the S-step scale. 0 is the oracle proper. */
#ifndef ORACLE_PLANT
#define ORACLE_PLANT 0
#endif

enum { O_OK = 0, O_EINVAL = 1, O_ENOTSPD = 2, O_EDIVERGED = 4, O_EMAXIT = 5, O_ENOMEM = 7 };

typedef struct {
  int n;
  int64_t nnz;
  int* rp;
  int* col;
  double* val;
} ocsr;

typedef struct {
  ocsr A, H, S; /* A copy, splitting on the union pattern */
  int split_ok; /* 1 if H == H^T and S == -S^T held bitwise */
} oracle_sys;

static void csr_free(ocsr* m) {
  free(m->rp);
  free(m->col);
  free(m->val);
  m->rp = NULL;
  m->col = NULL;
  m->val = NULL;
}

/* y = M x, one row at a time, left-to-right over the stored entries. */
static void spmv(const ocsr* M, const double* x, double* y) {
  int n = M->n;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int k = M->rp[i]; k < M->rp[i + 1]; ++k) s += M->val[k] * x[M->col[k]];
    y[i] = s;
  }
}

static double dot(int n, const double* a, const double* b) {
  double part[ORACLE_CHUNKS];
#pragma omp parallel for schedule(static)
  for (int c = 0; c < ORACLE_CHUNKS; ++c) {
    int64_t lo = (int64_t)n * c / ORACLE_CHUNKS, hi = (int64_t)n * (c + 1) / ORACLE_CHUNKS;
    double s = 0.0;
    for (int64_t i = lo; i < hi; ++i) s += a[i] * b[i];
    part[c] = s;
  }
  double s = 0.0;
  for (int c = 0; c < ORACLE_CHUNKS; ++c) s += part[c];
  return s;
}

/* Explicit CSR transpose (columns of the result come out sorted). */
static int transpose(const ocsr* A, ocsr* T) {
  int n = A->n;
  int64_t nnz = A->nnz;
  T->n = n;
  T->nnz = nnz;
  T->rp = (int*)calloc((size_t)n + 1, sizeof(int));
  T->col = (int*)malloc((size_t)(nnz ? nnz : 1) * sizeof(int));
  T->val = (double*)malloc((size_t)(nnz ? nnz : 1) * sizeof(double));
  if (!T->rp || !T->col || !T->val) return O_ENOMEM;
  for (int64_t k = 0; k < nnz; ++k) T->rp[A->col[k] + 1]++;
  for (int i = 0; i < n; ++i) T->rp[i + 1] += T->rp[i];
  int* next = (int*)malloc((size_t)n * sizeof(int) + 1);
  if (!next) return O_ENOMEM;
  memcpy(next, T->rp, (size_t)n * sizeof(int));
  for (int i = 0; i < n; ++i)
    for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
      int j = A->col[k];
      int dst = next[j]++;
      T->col[dst] = i;
      T->val[dst] = A->val[k];
    }
  free(next);
  return O_OK;
}

/* Merge rows of A and A^T (both column-sorted, duplicates summed) into
 * H = (A + A^T)/2 and S = (A - A^T)/2 on the union pattern. */
static int hss_split(const ocsr* A, const ocsr* At, ocsr* H, ocsr* S) {
  int n = A->n;
  int64_t cap = A->nnz + At->nnz;
  H->n = S->n = n;
  H->rp = (int*)calloc((size_t)n + 1, sizeof(int));
  S->rp = (int*)calloc((size_t)n + 1, sizeof(int));
  H->col = (int*)malloc((size_t)(cap ? cap : 1) * sizeof(int));
  S->col = (int*)malloc((size_t)(cap ? cap : 1) * sizeof(int));
  H->val = (double*)malloc((size_t)(cap ? cap : 1) * sizeof(double));
  S->val = (double*)malloc((size_t)(cap ? cap : 1) * sizeof(double));
  if (!H->rp || !S->rp || !H->col || !S->col || !H->val || !S->val) return O_ENOMEM;
  int64_t pos = 0;
  for (int i = 0; i < n; ++i) {
    int ka = A->rp[i], ea = A->rp[i + 1], kt = At->rp[i], et = At->rp[i + 1];
    while (ka < ea || kt < et) {
      int ca = ka < ea ? A->col[ka] : n;
      int ct = kt < et ? At->col[kt] : n;
      int c = ca < ct ? ca : ct;
      double va = 0.0, vt = 0.0;
      while (ka < ea && A->col[ka] == c) va += A->val[ka++];
      while (kt < et && At->col[kt] == c) vt += At->val[kt++];
      H->col[pos] = S->col[pos] = c;
      H->val[pos] = (va + vt) / 2.0;
      S->val[pos] = (va - vt) / 2.0;
      ++pos;
    }
    H->rp[i + 1] = S->rp[i + 1] = (int)pos;
  }
  H->nnz = S->nnz = pos;
  return O_OK;
}

/* Bitwise symmetry check: M(i,j) == sign * M(j,i) for every stored entry. */
static int check_sym(const ocsr* M, double sign) {
  for (int i = 0; i < M->n; ++i)
    for (int k = M->rp[i]; k < M->rp[i + 1]; ++k) {
      int j = M->col[k];
      /* binary search for (j, i) */
      int lo = M->rp[j], hi = M->rp[j + 1] - 1, found = -1;
      while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (M->col[mid] == i) {
          found = mid;
          break;
        }
        if (M->col[mid] < i) lo = mid + 1;
        else hi = mid - 1;
      }
      if (found < 0) return 0;
      if (M->val[k] != sign * M->val[found]) return 0;
    }
  return 1;
}

void oracle_free(oracle_sys* s) {
  if (!s) return;
  csr_free(&s->A);
  csr_free(&s->H);
  csr_free(&s->S);
  free(s);
}

/* Validate and copy A, form A^T, H and S.  Returns NULL on a malformed CSR. */
oracle_sys* oracle_setup(int n, const int* rp, const int* col, const double* val) {
  if (n < 1 || !rp || rp[0] != 0) return NULL;
  for (int i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return NULL;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      if (col[k] < 0 || col[k] >= n) return NULL;
      if (k > rp[i] && col[k] <= col[k - 1]) return NULL; /* sorted, unique */
    }
  }
  oracle_sys* s = (oracle_sys*)calloc(1, sizeof(oracle_sys));
  if (!s) return NULL;
  int64_t nnz = rp[n];
  s->A.n = n;
  s->A.nnz = nnz;
  s->A.rp = (int*)malloc(((size_t)n + 1) * sizeof(int));
  s->A.col = (int*)malloc((size_t)(nnz ? nnz : 1) * sizeof(int));
  s->A.val = (double*)malloc((size_t)(nnz ? nnz : 1) * sizeof(double));
  if (!s->A.rp || !s->A.col || !s->A.val) {
    oracle_free(s);
    return NULL;
  }
  memcpy(s->A.rp, rp, ((size_t)n + 1) * sizeof(int));
  memcpy(s->A.col, col, (size_t)nnz * sizeof(int));
  memcpy(s->A.val, val, (size_t)nnz * sizeof(double));
  ocsr At = {0};
  if (transpose(&s->A, &At) != O_OK || hss_split(&s->A, &At, &s->H, &s->S) != O_OK) {
    csr_free(&At);
    oracle_free(s);
    return NULL;
  }
  csr_free(&At);
  s->split_ok = check_sym(&s->H, 1.0) && check_sym(&s->S, -1.0);
  return s;
}

int oracle_split_ok(const oracle_sys* s) { return s->split_ok; }
int64_t oracle_split_nnz(const oracle_sys* s) { return s->H.nnz; }

/* Copy out H (which = 1) or S (which = 2) in CSR; arrays sized n+1 / split nnz. */
int oracle_get_split(const oracle_sys* s, int which, int* rp, int* col, double* val) {
  const ocsr* M = which == 1 ? &s->H : which == 2 ? &s->S : NULL;
  if (!M) return O_EINVAL;
  memcpy(rp, M->rp, ((size_t)M->n + 1) * sizeof(int));
  memcpy(col, M->col, (size_t)M->nnz * sizeof(int));
  memcpy(val, M->val, (size_t)M->nnz * sizeof(double));
  return O_OK;
}

/* y = M x for M = A (0), H (1) or S (2). */
int oracle_spmv(const oracle_sys* s, int which, const double* x, double* y) {
  const ocsr* M = which == 0 ? &s->A : which == 1 ? &s->H : which == 2 ? &s->S : NULL;
  if (!M) return O_EINVAL;
  spmv(M, x, y);
  return O_OK;
}

/* Operators of the two inner systems. */
typedef struct {
  const oracle_sys* s;
  double alpha;
  double* tmp;
} op_ctx;

/* q = (alpha I + H) p */
static void apply_h(const op_ctx* c, const double* p, double* q) {
  int n = c->s->H.n;
  spmv(&c->s->H, p, q);
  for (int i = 0; i < n; ++i) q[i] = c->alpha * p[i] + q[i];
}

/* q = (alpha^2 I - S^2) p = (alpha I + S)(alpha I - S) p */
static void apply_s_normal(const op_ctx* c, const double* p, double* q) {
  int n = c->s->S.n;
  spmv(&c->s->S, p, c->tmp);
  spmv(&c->s->S, c->tmp, q);
  double a2 = c->alpha * c->alpha;
  for (int i = 0; i < n; ++i) q[i] = a2 * p[i] - q[i];
}

/* Conjugate gradients (Hestenes-Stiefel) from a zero start for an SPD
 * operator; stops when ||g - K z||_2 <= eps ||g||_2 (recurrence residual) or
 * after maxit steps.  Returns the step count, -1 on a non-positive curvature. */
static int cg(void (*apply)(const op_ctx*, const double*, double*), const op_ctx* c, int n,
              const double* g, double* z, double eps, int maxit, double* r, double* p, double* q) {
  for (int i = 0; i < n; ++i) {
    z[i] = 0.0;
    r[i] = g[i];
    p[i] = g[i];
  }
  double rr = dot(n, r, r);
  double stop = eps * eps * rr;
  if (rr == 0.0) return 0;
  int it = 0;
  while (it < maxit) {
    apply(c, p, q);
    double pq = dot(n, p, q);
    if (!(pq > 0.0)) return -1;
    double a = rr / pq;
    for (int i = 0; i < n; ++i) {
      z[i] += a * p[i];
      r[i] -= a * q[i];
    }
    double rr_new = dot(n, r, r);
    ++it;
    if (rr_new <= stop) break;
    double b = rr_new / rr;
    for (int i = 0; i < n; ++i) p[i] = r[i] + b * p[i];
    rr = rr_new;
  }
  return it;
}

/*
 * GADI-IR in double.  x holds x_0 on entry (the paper's experiments use 0)
 * and the last iterate on return.  Outputs: sweeps = corrections applied,
 * inner step totals, final RES = ||r||/||r_0||; hist[k] = RES before sweep k
 * (up to hist_len entries).  Status: 0 converged, 4 diverged (non-finite or
 * ||r|| > 1e6 ||r_0||), 5 sweep limit, 2 non-SPD inner operator, 1 bad args.
 */
int oracle_gadi(const oracle_sys* s, const double* b, double* x, double alpha, double omega,
                double tol, double eps_h, double eps_s, int maxit_out, int maxit_in, int* sweeps,
                int64_t* inner_h, int64_t* inner_s, double* relres, double* hist, int hist_len) {
  if (!(alpha > 0.0) || !(omega >= 0.0 && omega < 2.0) || !(tol >= 0.0)) return O_EINVAL;
  int n = s->A.n;
  double* w = (double*)malloc((size_t)n * 9 * sizeof(double));
  if (!w) return O_ENOMEM;
  double *r = w, *z = w + n, *g = w + 2 * (size_t)n, *y = w + 3 * (size_t)n;
  double *t1 = w + 4 * (size_t)n, *t2 = w + 5 * (size_t)n, *t3 = w + 6 * (size_t)n;
  double *tmp = w + 7 * (size_t)n, *wv = w + 8 * (size_t)n;
  op_ctx c = {s, alpha, tmp};
#if ORACLE_PLANT == 2
  double p_scale = (1.0 - omega) * alpha;
#else
  double p_scale = (2.0 - omega) * alpha;
#endif
  double rho0 = 0.0;
  int status = O_EMAXIT;
  int k = 0;
  *inner_h = 0;
  *inner_s = 0;
  for (;; ++k) {
    /* step 1: r = b - A x */
    spmv(&s->A, x, r);
    for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double rho = sqrt(dot(n, r, r));
    if (k == 0) rho0 = rho;
    double res = rho0 > 0.0 ? rho / rho0 : 0.0;
    if (k < hist_len) hist[k] = res;
    *relres = res;
    if (rho <= tol * rho0) {
      status = O_OK;
      break;
    }
    if (!isfinite(rho) || rho > 1e6 * rho0) {
      status = O_EDIVERGED;
      break;
    }
    if (k == maxit_out) {
      status = O_EMAXIT;
      break;
    }
    /* step 2: (alpha I + H) z = r */
    int ih = cg(apply_h, &c, n, r, z, eps_h, maxit_in, t1, t2, t3);
    if (ih < 0) {
      status = O_ENOTSPD;
      break;
    }
    *inner_h += ih;
    /* step 3: (alpha I + S) y = (2 - omega) alpha z via CGNE */
    for (int i = 0; i < n; ++i) g[i] = p_scale * z[i];
    int is = cg(apply_s_normal, &c, n, g, wv, eps_s, maxit_in, t1, t2, t3);
    if (is < 0) {
      status = O_ENOTSPD;
      break;
    }
    *inner_s += is;
    spmv(&s->S, wv, y);
#if ORACLE_PLANT == 1
    for (int i = 0; i < n; ++i) y[i] = alpha * wv[i] + y[i];
#else
    for (int i = 0; i < n; ++i) y[i] = alpha * wv[i] - y[i];
#endif
    /* step 4: x = x + y */
    for (int i = 0; i < n; ++i) x[i] += y[i];
  }
  *sweeps = k;
  free(w);
  return status;
}

/* Gershgorin data of the splitting: out[0] = min_i (H_ii - R_i^H),
 * out[1] = max_i (H_ii + R_i^H), out[2] = max_i R_i^S, out[3] = min_i R_i^S,
 * with R_i the off-diagonal absolute row sum. */
int oracle_gershgorin(const oracle_sys* s, double* out) {
  double hmin = INFINITY, hmax = -INFINITY, smax = -INFINITY, smin = INFINITY;
  for (int i = 0; i < s->H.n; ++i) {
    double d = 0.0, rh = 0.0, rs = 0.0;
    for (int k = s->H.rp[i]; k < s->H.rp[i + 1]; ++k) {
      if (s->H.col[k] == i) d = s->H.val[k];
      else rh += fabs(s->H.val[k]);
    }
    for (int k = s->S.rp[i]; k < s->S.rp[i + 1]; ++k)
      if (s->S.col[k] != i) rs += fabs(s->S.val[k]);
    if (d - rh < hmin) hmin = d - rh;
    if (d + rh > hmax) hmax = d + rh;
    if (rs > smax) smax = rs;
    if (rs < smin) smin = rs;
  }
  out[0] = hmin;
  out[1] = hmax;
  out[2] = smax;
  out[3] = smin;
  return O_OK;
}

/* Sets the threads of the OpenMP loops (no effect without OpenMP). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* Threads the OpenMP loops of the oracle use (1 without OpenMP). */
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
