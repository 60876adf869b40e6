/*
 * oracle.h -- plain CPU FP64 reference for the two band reductions.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the HIP path.
 *
 * Both routines are the unblocked (one column at a time) Householder
 * reductions.  The blocked algorithm of the paper (Sec. 2.1, eqs. updateA0 to
 * updateA2syr2k; Sec. 3.1, eqs. updateB to updateD) reaches the same result up
 * to rounding whenever the block size b does not exceed the bandwidth w,
 * because no reflector of a block touches another column of the same panel
 * from the right.  The oracle is therefore the b = 1 case.
 *
 * Storage: column-major, leading dimension lda, FP64, host memory.
 * Return: 0 on success, -i when argument i is invalid (LAPACK info style).
 */
#ifndef BANDRED_ORACLE_H
#define BANDRED_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Symmetric n x n matrix (lower triangle referenced and written) to symmetric
 * band form of bandwidth w (Sec. 2.1).  Processes reflector columns
 * c = 0 .. min(ncols, n-w-1)-1; ncols < 0 means all of them.  On return the
 * band (0 <= i-j <= w) holds B, column c holds v[1:] of reflector c in rows
 * c+w+1 .. n-1 (v[0] = 1 implicit at row c+w), and tau[c] its scalar.
 * tau has n-w entries when n > w (tau[n-w-1] = 0); it is unused otherwise. */
int oracle_sy2sb(int64_t n, int64_t w, int64_t ncols, double *A, int64_t lda,
                 double *tau);

/* General m x n matrix, m >= n, to upper triangular-band form with upper
 * bandwidth w (Sec. 3.1).  Processes steps c = 0 .. min(ncols, n)-1
 * (ncols < 0: all).  Step c: left reflector of column c (rows c..m-1, stored
 * below the diagonal, scalar tauq[c]); then, if c <= n-w-2, right reflector of
 * row c (columns c+w..n-1, stored right of entry (c, c+w), scalar taup[c]).
 * tauq and taup have n entries each; entries with no reflector are 0. */
int oracle_ge2gb(int64_t m, int64_t n, int64_t w, int64_t ncols, double *A,
                 int64_t lda, double *tauq, double *taup);

/* General m x n matrix, m >= n, to band form with lower AND upper bandwidth w
 * (Sec. 3.3).  Processes steps c = 0 .. min(ncols, n)-1 (ncols < 0: all).
 * Step c: left reflector of column c acting on rows c+w..m-1 (beta at
 * (c+w, c), v[1:] below it, scalar tauq[c]; only when c+w < m), then right
 * reflector of row c acting on columns c+w..n-1 (gamma at (c, c+w), u[1:] to
 * its right, scalar taup[c]; only when c+w < n).  tauq and taup have n
 * entries each; entries with no reflector (or a length-1 one) are 0.  On
 * return B(i,j) for -w <= j-i <= w holds the band; U = H_0 H_1 ...,
 * V = G_0 G_1 ..., B = U^T A V. */
int oracle_ge2gb_lu(int64_t m, int64_t n, int64_t w, int64_t ncols, double *A,
                    int64_t lda, double *tauq, double *taup);

/* C := Q C (trans = 0) or Q^T C (trans = 1) for Q = H_0 H_1 ... H_{nrefl-1}
 * made of stored reflectors (back-transformation).  Reflector i acts on
 * indices i+off .. len-1; its vector has v[0] = 1 implicit at index i+off
 * and v[t], t >= 1, at A(i+off+t, i) (rowstore = 0) or A(i, i+off+t)
 * (rowstore = 1); tau[i] its scalar.  C is len x k, column-major, ld ldc.
 *   sy2sb Q:      rowstore 0, off w, nrefl n-w, len n
 *   ge2gb U:      rowstore 0, off 0, nrefl n, len m
 *   ge2gb V:      rowstore 1, off w, nrefl max(0, n-w), len n
 *   ge2gb_lu U:   rowstore 0, off w, nrefl min(n, max(0, m-w)), len m
 *   ge2gb_lu V:   rowstore 1, off w, nrefl max(0, n-w), len n */
int oracle_apply_refl(int rowstore, int64_t off, int64_t nrefl, int64_t len,
                      const double *A, int64_t lda, const double *tau, int trans,
                      int64_t k, double *C, int64_t ldc);

/* All eigenvalues (ascending) of the n x n symmetric tridiagonal matrix with
 * diagonal d (n entries) and off-diagonal e (n-1 entries), by bisection on
 * the Sturm count (number of negative pivots of LDL^T of T - x I), each
 * interval halved until its ends are adjacent doubles.  The eigenvalue step
 * after the band and tridiagonal reductions (the paper's pipeline ends with
 * LAPACK's DSTERF, Sec. 4.3). */
int oracle_tridiag_eigvals(int64_t n, const double *d, const double *e, double *lam);

/* Householder vector of x (length L, stride inc): on return x[0] is left
 * alone, x[1:] holds v[1:], *beta the new leading entry; returns tau. */
double oracle_house(int64_t L, double *x, int64_t inc, double *beta);

/* Number of OpenMP threads the oracle uses. */
int oracle_threads(void);

/* Set the number of OpenMP threads for later calls (results do not depend
 * on it; used to time the oracle single-threaded). */
void oracle_set_threads(int nthreads);

#ifdef __cplusplus
}
#endif
#endif
