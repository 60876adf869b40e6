/*
 * oracle.c -- plain CPU FP64 reference for the reduction of a dense matrix to
 * compact band form (Rodriguez-Sanchez, Catalan, Herrero, Quintana-Orti,
 * Tomas: look-ahead in the two-sided reduction to compact band forms).
 *
 * TEST INFRASTRUCTURE ONLY.  It exists to check the HIP implementation; the
 * product library never links, loads or calls it, and the two share no
 * source.  Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math), so every
 * product and sum is rounded once, in IEEE double, in program order.
 *
 * What it computes (see oracle.h for the storage contract):
 *   - sy2sb: Sec. 2.1.  Each reflector H = I - tau v v^T annihilates column c
 *     below row c+w; the similarity H A2 H of the trailing block uses the
 *     symmetric rank-2 form of eqs. updateA2symm..updateA2syr2k taken at block
 *     size 1 (p = tau A2 v, K = tau p^T v / 2, q = p - K v,
 *     A2 -= v q^T + q v^T); the in-band columns between the reflector column
 *     and the trailing block only see H from the left (eq. updateA1).
 *   - ge2gb: Sec. 3.1, eqs. updateB..updateD at block size 1: a left
 *     reflector annihilates column c below the diagonal and is applied from
 *     the left to the columns right of it; a right reflector annihilates
 *     row c right of column c+w and is applied from the right to the rows
 *     below it.
 *   - The reflector itself is the textbook Householder vector (Golub and Van
 *     Loan, the reference the paper cites for the WY machinery): with
 *     alpha = x0, sigma = ||x[1:]||, beta = -sign(alpha) hypot(alpha, sigma),
 *     tau = (beta - alpha) / beta, v = [1; x[1:] / (alpha - beta)], and
 *     tau = 0, beta = alpha when sigma = 0.  sign(+-0) = +1.
 *
 * Parallelism: OpenMP over independent columns (or row chunks) only; every
 * sum is accumulated by one thread in a fixed order, so results do not depend
 * on the thread count.
 *
 * Also: ge2gb_lu (Sec. 3.3, band form with equal lower and upper bandwidth,
 * eqs. updateB0..updateCD22 at block size 1) and apply_refl (the product of
 * the stored reflectors applied to a matrix, the back-transformation).
 *
 * ORACLE_MUTANT (compile-time, default 0) plants one deliberate mistake; the
 * test-suite builds such variants to show that its pins catch them.  A normal
 * build never defines it.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

/* Euclidean norm of x[0..L-1] (stride inc), scaled by max |x_i| so that the
 * squares neither overflow nor underflow. */
static double norm2_scaled(int64_t L, const double *x, int64_t inc) {
  double m = 0.0;
  for (int64_t i = 0; i < L; ++i) {
    double a = fabs(x[i * inc]);
    if (a > m) m = a;
  }
  if (m == 0.0) return 0.0;
  double s = 0.0;
  for (int64_t i = 0; i < L; ++i) {
    double t = x[i * inc] / m;
    s += t * t;
  }
  return m * sqrt(s);
}

double oracle_house(int64_t L, double *x, int64_t inc, double *beta) {
  double alpha = x[0];
  if (L <= 1) {
    *beta = alpha;
    return 0.0;
  }
  double sigma = norm2_scaled(L - 1, x + inc, inc);
  if (sigma == 0.0) {
    *beta = alpha;
    return 0.0;
  }
  double s = (alpha < 0.0) ? -1.0 : 1.0;
#if ORACLE_MUTANT == 2
  double b = s * hypot(alpha, sigma); /* planted: wrong sign of beta */
#else
  double b = -s * hypot(alpha, sigma);
#endif
  double tau = (b - alpha) / b;
  double d = alpha - b;
  for (int64_t i = 1; i < L; ++i) x[i * inc] = x[i * inc] / d;
  *beta = b;
  return tau;
}

/* ------------------------------------------------------------------------ */
/* Symmetric band reduction                                                  */
/* ------------------------------------------------------------------------ */

int oracle_sy2sb(int64_t n, int64_t w, int64_t ncols, double *A, int64_t lda,
                 double *tau) {
  if (n < 0) return -1;
  if (w < 1) return -2;
  if (n > 0 && A == NULL) return -4;
  if (lda < (n > 1 ? n : 1)) return -5;
  if (n > w && tau == NULL) return -6;
  if (n <= w) return 0;

  for (int64_t c = 0; c < n - w; ++c) tau[c] = 0.0;
  int64_t nref = n - w - 1; /* reflector columns c = 0 .. n-w-2 */
  if (ncols >= 0 && ncols < nref) nref = ncols;
  if (nref <= 0) return 0;

  /* Full symmetric working copy S (n x n, column-major, ld n): the lower
   * triangle of A mirrored.  The rank-2 update below keeps it exactly
   * symmetric, so A2 v can be formed as column dots. */
  double *S = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
  double *v = (double *)malloc(sizeof(double) * (size_t)n);
  double *p = (double *)malloc(sizeof(double) * (size_t)n);
  double *q = (double *)malloc(sizeof(double) * (size_t)n);
  if (!S || !v || !p || !q) {
    free(S); free(v); free(p); free(q);
    return 2;
  }
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = j; i < n; ++i) {
      S[i + j * n] = A[i + j * lda];
      S[j + i * n] = A[i + j * lda];
    }

  for (int64_t c = 0; c < nref; ++c) {
    const int64_t r = c + w;   /* first row of the reflector */
    const int64_t L = n - r;   /* its length */
    double beta;
    double tc = oracle_house(L, S + r + c * n, 1, &beta);
    v[0] = 1.0;
    for (int64_t i = 1; i < L; ++i) v[i] = S[r + i + c * n];

    if (tc != 0.0) {
      double *A2 = S + r + r * n; /* trailing block, ld n */
      /* p = tau * A2 v */
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < L; ++i) {
        const double *col = A2 + i * n;
        double s = 0.0;
#if ORACLE_MUTANT == 4
        for (int64_t k = 1; k < L; ++k) s += col[k] * v[k]; /* planted: v[0] dropped */
#else
        for (int64_t k = 0; k < L; ++k) s += col[k] * v[k];
#endif
        p[i] = tc * s;
      }
      /* K = tau/2 * p^T v ; q = p - K v */
      double pv = 0.0;
      for (int64_t i = 0; i < L; ++i) pv += p[i] * v[i];
#if ORACLE_MUTANT == 1
      double K = tc * pv; /* planted: the factor 1/2 dropped */
#else
      double K = 0.5 * tc * pv;
#endif
      for (int64_t i = 0; i < L; ++i) q[i] = p[i] - K * v[i];
      /* A2 -= v q^T + q v^T  (both triangles, stays symmetric) */
#pragma omp parallel for schedule(static)
      for (int64_t k = 0; k < L; ++k) {
        double *col = A2 + k * n;
        const double vk = v[k], qk = q[k];
        for (int64_t i = 0; i < L; ++i) col[i] -= v[i] * qk + q[i] * vk;
      }
#if ORACLE_MUTANT != 3
      /* in-band columns c+1 .. r-1: H from the left only, rows r .. n-1 */
#pragma omp parallel for schedule(static)
      for (int64_t j = c + 1; j < r; ++j) {
        double *col = S + r + j * n;
        double s = 0.0;
        for (int64_t i = 0; i < L; ++i) s += v[i] * col[i];
        const double f = tc * s;
        for (int64_t i = 0; i < L; ++i) {
          col[i] -= f * v[i];
          S[j + (r + i) * n] = col[i];
        }
      }
#endif
    }
    S[r + c * n] = beta;
    tau[c] = tc;
  }

#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = j; i < n; ++i) A[i + j * lda] = S[i + j * n];

  free(S); free(v); free(p); free(q);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* General matrix to upper triangular-band                                   */
/* ------------------------------------------------------------------------ */

int oracle_ge2gb(int64_t m, int64_t n, int64_t w, int64_t ncols, double *A,
                 int64_t lda, double *tauq, double *taup) {
  if (m < 0) return -1;
  if (n < 0) return -2;
  if (m < n) return -1;
  if (w < 1) return -3;
  if (n > 0 && A == NULL) return -5;
  if (lda < (m > 1 ? m : 1)) return -6;
  if (n > 0 && tauq == NULL) return -7;
  if (n > 0 && taup == NULL) return -8;
  if (n == 0) return 0;

  for (int64_t c = 0; c < n; ++c) tauq[c] = taup[c] = 0.0;
  int64_t nsteps = n;
  if (ncols >= 0 && ncols < nsteps) nsteps = ncols;

  double *u = (double *)malloc(sizeof(double) * (size_t)(m > n ? m : n));
  double *s = (double *)malloc(sizeof(double) * (size_t)m);
  if (!u || !s) {
    free(u); free(s);
    return 2;
  }

  for (int64_t c = 0; c < nsteps; ++c) {
    /* left reflector: column c, rows c .. m-1 */
    {
      const int64_t L = m - c;
      double beta;
      double tq = oracle_house(L, A + c + c * lda, 1, &beta);
      u[0] = 1.0;
      for (int64_t i = 1; i < L; ++i) u[i] = A[c + i + c * lda];
      if (tq != 0.0) {
#if ORACLE_MUTANT == 6
        const int64_t jend = (c + w < n) ? c + w : n; /* planted: far columns skipped */
#else
        const int64_t jend = n;
#endif
#pragma omp parallel for schedule(static)
        for (int64_t j = c + 1; j < jend; ++j) {
          double *col = A + c + j * lda;
          double d = 0.0;
          for (int64_t i = 0; i < L; ++i) d += u[i] * col[i];
          const double f = tq * d;
          for (int64_t i = 0; i < L; ++i) col[i] -= f * u[i];
        }
      }
      A[c + c * lda] = beta;
      tauq[c] = tq;
    }
    /* right reflector: row c, columns c+w .. n-1 */
    if (c <= n - w - 2) {
      const int64_t c0 = c + w;
      const int64_t L = n - c0;
      double gamma;
      double tp = oracle_house(L, A + c + c0 * lda, lda, &gamma);
      u[0] = 1.0;
      for (int64_t k = 1; k < L; ++k) u[k] = A[c + (c0 + k) * lda];
      if (tp != 0.0) {
#if ORACLE_MUTANT == 5
        const int64_t r0 = c; /* planted: row c itself updated */
#else
        const int64_t r0 = c + 1;
#endif
        const int64_t nr = m - r0;
        int nt = oracle_threads();
        int64_t chunk = (nr + nt - 1) / nt;
        if (chunk < 64) chunk = 64;
#pragma omp parallel for schedule(static)
        for (int64_t r1 = 0; r1 < nr; r1 += chunk) {
          const int64_t r2 = (r1 + chunk < nr) ? r1 + chunk : nr;
          double *sr = s + r0;
          for (int64_t r = r1; r < r2; ++r) sr[r] = 0.0;
          for (int64_t k = 0; k < L; ++k) {
            const double *col = A + r0 + (c0 + k) * lda;
            const double uk = u[k];
            for (int64_t r = r1; r < r2; ++r) sr[r] += col[r] * uk;
          }
          for (int64_t k = 0; k < L; ++k) {
            double *col = A + r0 + (c0 + k) * lda;
            const double f = tp * u[k];
            for (int64_t r = r1; r < r2; ++r) col[r] -= sr[r] * f;
          }
        }
      }
      A[c + c0 * lda] = gamma;
      taup[c] = tp;
    }
  }
  free(u); free(s);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* General matrix to band form with equal lower and upper bandwidth         */
/* ------------------------------------------------------------------------ */

/* Sec. 3.3 (eqs. updateB0..updateCD22) at block size 1.  Step c: the left
 * reflector of column c annihilates rows c+w+1 .. m-1 of that column and is
 * applied from the left to the columns right of it (rows c+w .. m-1); the
 * right reflector of row c annihilates columns c+w+1 .. n-1 of that row and
 * is applied from the right to the rows below it (columns c+w .. n-1).  The
 * two reflectors of one step touch disjoint parts of each other's vector
 * (rows >= c+w versus row c, columns >= c+w versus column c), so their order
 * within a step does not matter; the left one is taken first. */
int oracle_ge2gb_lu(int64_t m, int64_t n, int64_t w, int64_t ncols, double *A,
                    int64_t lda, double *tauq, double *taup) {
  if (m < 0) return -1;
  if (n < 0) return -2;
  if (m < n) return -1;
  if (w < 1) return -3;
  if (n > 0 && A == NULL) return -5;
  if (lda < (m > 1 ? m : 1)) return -6;
  if (n > 0 && tauq == NULL) return -7;
  if (n > 0 && taup == NULL) return -8;
  if (n == 0) return 0;

  for (int64_t c = 0; c < n; ++c) tauq[c] = taup[c] = 0.0;
  int64_t nsteps = n;
  if (ncols >= 0 && ncols < nsteps) nsteps = ncols;

  double *u = (double *)malloc(sizeof(double) * (size_t)(m > n ? m : n));
  double *s = (double *)malloc(sizeof(double) * (size_t)m);
  if (!u || !s) {
    free(u); free(s);
    return 2;
  }

  for (int64_t c = 0; c < nsteps; ++c) {
    /* left reflector: column c, rows c+w .. m-1 */
    const int64_t r = c + w;
    if (r < m) {
      const int64_t L = m - r;
      double beta;
      double tq = oracle_house(L, A + r + c * lda, 1, &beta);
      u[0] = 1.0;
      for (int64_t i = 1; i < L; ++i) u[i] = A[r + i + c * lda];
      if (tq != 0.0) {
#if ORACLE_MUTANT == 8
        const int64_t j0 = (c + w < n) ? c + w : n; /* planted: in-band columns skipped */
#else
        const int64_t j0 = c + 1;
#endif
#pragma omp parallel for schedule(static)
        for (int64_t j = j0; j < n; ++j) {
          double *col = A + r + j * lda;
          double d = 0.0;
          for (int64_t i = 0; i < L; ++i) d += u[i] * col[i];
          const double f = tq * d;
          for (int64_t i = 0; i < L; ++i) col[i] -= f * u[i];
        }
      }
      A[r + c * lda] = beta;
      tauq[c] = tq;
    }
    /* right reflector: row c, columns c+w .. n-1 */
    const int64_t c0 = c + w;
    if (c0 < n) {
      const int64_t L = n - c0;
      double gamma;
      double tp = oracle_house(L, A + c + c0 * lda, lda, &gamma);
      u[0] = 1.0;
      for (int64_t k = 1; k < L; ++k) u[k] = A[c + (c0 + k) * lda];
      if (tp != 0.0) {
#if ORACLE_MUTANT == 7
        const int64_t r0 = (c + w < m) ? c + w : m; /* planted: rows c+1..c+w-1 skipped */
#else
        const int64_t r0 = c + 1;
#endif
        const int64_t nr = m - r0;
        int nt = oracle_threads();
        int64_t chunk = (nr + nt - 1) / nt;
        if (chunk < 64) chunk = 64;
#pragma omp parallel for schedule(static)
        for (int64_t r1 = 0; r1 < nr; r1 += chunk) {
          const int64_t r2 = (r1 + chunk < nr) ? r1 + chunk : nr;
          double *sr = s + r0;
          for (int64_t q = r1; q < r2; ++q) sr[q] = 0.0;
          for (int64_t k = 0; k < L; ++k) {
            const double *col = A + r0 + (c0 + k) * lda;
            const double uk = u[k];
            for (int64_t q = r1; q < r2; ++q) sr[q] += col[q] * uk;
          }
          for (int64_t k = 0; k < L; ++k) {
            double *col = A + r0 + (c0 + k) * lda;
            const double f = tp * u[k];
            for (int64_t q = r1; q < r2; ++q) col[q] -= sr[q] * f;
          }
        }
      }
      A[c + c0 * lda] = gamma;
      taup[c] = tp;
    }
  }
  free(u); free(s);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Applying the stored reflectors (back-transformation)                      */
/* ------------------------------------------------------------------------ */

/* The orthogonal factor of a reduction is the product of its reflectors
 * taken in the order they were made, Q = H_0 H_1 ... H_{nrefl-1} (Sec. 2.1
 * and Sec. 3: Q is accumulated as I + W Y^T panel by panel).  Reflector i acts
 * on indices i+off .. len-1 with v[0] = 1 at index i+off and v[t] (t >= 1)
 * stored at A(i+off+t, i) (column storage) or A(i, i+off+t) (row storage).
 * trans = 0: C := Q C; trans = 1: C := Q^T C = H_{nrefl-1} ... H_0 C, for the
 * len x k matrix C (ld ldc).  One reflector at a time, each column of C on its
 * own (OpenMP over the columns of C). */
int oracle_apply_refl(int rowstore, int64_t off, int64_t nrefl, int64_t len,
                      const double *A, int64_t lda, const double *tau, int trans,
                      int64_t k, double *C, int64_t ldc) {
  if (off < 0) return -2;
  if (nrefl < 0 || nrefl + off > len) return -3;
  if (len < 0) return -4;
  if (nrefl > 0 && A == NULL) return -5;
  if (nrefl > 0 && tau == NULL) return -7;
  if (trans != 0 && trans != 1) return -8;
  if (k < 0) return -9;
  if (k > 0 && len > 0 && C == NULL) return -10;
  if (ldc < (len > 1 ? len : 1)) return -11;
  if (nrefl == 0 || k == 0) return 0;
  double *v = (double *)malloc(sizeof(double) * (size_t)len);
  if (!v) return 2;
  for (int64_t step = 0; step < nrefl; ++step) {
#if ORACLE_MUTANT == 9
    const int64_t i = step; /* planted: Q C applied in the order of Q^T C */
    (void)trans;
#else
    const int64_t i = trans ? step : nrefl - 1 - step;
#endif
    const double t = tau[i];
    if (t == 0.0) continue;
    const int64_t r = i + off, L = len - r;
    v[0] = 1.0;
    for (int64_t q = 1; q < L; ++q)
      v[q] = rowstore ? A[i + (r + q) * lda] : A[(r + q) + i * lda];
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < k; ++j) {
      double *col = C + r + j * ldc;
      double d = 0.0;
      for (int64_t q = 0; q < L; ++q) d += v[q] * col[q];
      const double f = t * d;
      for (int64_t q = 0; q < L; ++q) col[q] -= f * v[q];
    }
  }
  free(v);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Eigenvalues of a symmetric tridiagonal matrix (the last step of the       */
/* two-stage eigenvalue pipeline that follows the band reduction)            */
/* ------------------------------------------------------------------------ */

/* Number of eigenvalues of T = tridiag(e, d, e) smaller than x: the number of
 * negative pivots of the LDL^T factorisation of T - x I (Sylvester's law of
 * inertia; the Sturm sequence count of Golub and Van Loan, Sec. 8.4).  A
 * pivot that is exactly zero is replaced by -pivmin, as if x had been moved by
 * a tiny amount. */
static int64_t sturm_count(int64_t n, const double *d, const double *e, double x,
                           double pivmin) {
  int64_t cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++cnt;
  for (int64_t i = 1; i < n; ++i) {
#if ORACLE_MUTANT == 10
    q = (d[i] - x) + e[i - 1] * e[i - 1] / q; /* planted: wrong sign of the update */
#else
    q = (d[i] - x) - e[i - 1] * e[i - 1] / q;
#endif
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

/* All eigenvalues of the n x n symmetric tridiagonal matrix with diagonal d
 * and off-diagonal e (n-1 entries), ascending, by bisection: eigenvalue k is
 * the point where the count of eigenvalues below x passes from <= k to > k.
 * The search starts from the Gershgorin interval and halves it until the two
 * ends are adjacent doubles (or equal). */
int oracle_tridiag_eigvals(int64_t n, const double *d, const double *e, double *lam) {
  if (n < 0) return -1;
  if (n > 0 && (d == NULL || lam == NULL)) return -2;
  if (n > 1 && e == NULL) return -3;
  if (n == 0) return 0;
  double lo = d[0], hi = d[0], emax2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0);
    if (d[i] - r < lo) lo = d[i] - r;
    if (d[i] + r > hi) hi = d[i] + r;
    if (i < n - 1 && e[i] * e[i] > emax2) emax2 = e[i] * e[i];
  }
  const double pivmin = 2.2250738585072014e-308 * (emax2 > 1.0 ? emax2 : 1.0);
  const double pad = 2.220446049250313e-16 * (fabs(lo) > fabs(hi) ? fabs(lo) : fabs(hi)) * 4.0 +
                     pivmin;
  lo -= pad;
  hi += pad;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < n; ++k) {
    double a = lo, b = hi;
    for (int it = 0; it < 2200; ++it) {
      const double mid = 0.5 * (a + b);
      if (mid <= a || mid >= b) break; /* a and b adjacent */
      if (sturm_count(n, d, e, mid, pivmin) > k) b = mid;
      else a = mid;
    }
    lam[k] = 0.5 * (a + b);
  }
  return 0;
}
