/*
 * bandred.h -- C ABI of the MI355X (gfx950) band-reduction library.
 *
 * The library computes the first stage of two-stage dense eigen- and
 * singular-value solvers: the blocked two-sided Householder reduction of
 *   - a dense symmetric matrix to symmetric band form with bandwidth w
 *     (Sec. 2.1 of Rodriguez-Sanchez et al., "Look-ahead in the two-sided
 *     reduction to compact band forms", eqs. updateA0 to updateA2syr2k), and
 *   - a dense general m x n matrix (m >= n) to upper triangular-band form with
 *     upper bandwidth w (Sec. 3.1, eqs. updateB to updateD).
 * b is the algorithmic block size (panel width), 1 <= b <= w (Sec. 2.1).
 *
 * Conventions shared by every entry point
 *   - Matrices are FP64, column-major, leading dimension lda (in elements).
 *   - Unless a name ends in _host, every matrix and tau pointer is a DEVICE
 *     pointer (HIP global memory on the current device).  The caller owns all
 *     of them; the library keeps no pointer after the call returns.
 *   - Reflectors use the LAPACK convention H = I - tau v v^T with v[0] = 1
 *     implicit; the product of the reflectors of one panel is I - V T V^T
 *     with T upper triangular (compact WY).  The paper writes Q = I + W Y^T;
 *     the two agree with Y = V and W = -V T.
 *   - The library allocates its own device workspace (cached per device and
 *     grown on demand).  Calls on the same device are ordered on that
 *     workspace: a call waits (on its stream) for the previous call's work.
 *   - Return value: 0 on success; -i when argument i (1-based) is invalid;
 *     a positive BANDRED_ERR_* code on a runtime failure.
 */
#ifndef BANDRED_H
#define BANDRED_H

#include <stdint.h>

#ifndef BANDRED_API
#define BANDRED_API __attribute__((visibility("default")))
#endif

#ifdef __cplusplus
extern "C" {
#endif

enum {
  BANDRED_OK = 0,
  BANDRED_ERR_HIP = 1,         /* a HIP runtime call failed */
  BANDRED_ERR_ALLOC = 2,       /* device workspace allocation failed */
  BANDRED_ERR_UNSUPPORTED = 3, /* device or problem shape not supported */
  BANDRED_ERR_TIMEOUT = 4      /* a kernel's bounded inter-workgroup wait gave up */
};

/* Arithmetic of the trailing-update products (the SYMM/SYR2K of eqs.
 * updateA2symm/updateA2syr2k, the left update of eq. updateA1 and the
 * GEMM pairs of eqs. updateCD/updateD).  Panels, tau and T are FP64 always. */
typedef enum {
  BANDRED_FP64 = 0,           /* FP64 MFMA, FP64 accumulation */
  BANDRED_FP32_UPDATE = 1,    /* operands rounded to FP32, FP32 MFMA and accumulation,
                                 result added to the FP64 matrix */
  BANDRED_SPLIT32_UPDATE = 2, /* x = hi + lo (both FP32); hi*hi + hi*lo + lo*hi on FP32
                                 MFMA with FP32 accumulation, summed in FP64 */
  BANDRED_INT8_SPLIT_UPDATE = 3 /* exact split (error-free slicing): each row of the left
                                 operand and column of the right one scaled by a power of
                                 two and cut into 7 signed base-256 int8 digits; the 28
                                 digit products of order <= 8 run on int8 MFMA with exact
                                 int32 sums and are combined in FP64.  Per term of the
                                 inner dimension the error is below 2^-49 of the product
                                 of the row's and the column's largest entries, under the
                                 worst-case error of an FP64 dot product.  Rank-2k updates
                                 scale their two halves apart.  A row or column holding a
                                 NaN or Inf makes every sum it enters NaN.  Not in the
                                 paper (which is FP64 throughout).  Work space grows by
                                 about 7 (n + 2w) n bytes (SY2SB; m and n for GE2GB) */
} bandred_prec_t;

/* Optional knobs for the _ex entry points (pass NULL for defaults). */
typedef struct {
  int lookahead;      /* 1 (default): factor the next panel on a second stream while
                         the rest of the trailing matrix is updated (Sec. 2.2);
                         0: one stream, strictly sequential (debug / comparison) */
  int panel_rows;     /* rows per workgroup of the per-column panel kernel; 0 = automatic */
  int panel_method;   /* 0 (default) or 2: CholeskyQR2 + Householder reconstruction, with the
                         per-column kernel as fallback for rank-deficient panels and
                         panels with a column that is zero below its diagonal;
                         1: per-column Householder kernel only */
  int update_chunks;  /* the split of the chip between a look-ahead panel and the update
                         beside it: an update that runs beside a panel is issued as at most
                         this many launches (1..8), between which CUs drain and a waiting
                         panel kernel takes one; each launch keeps at least two rounds of
                         resident workgroups.  0 (default): 3 for GEMM updates, 2 for the
                         SYR2K, or the autotuner's choice when b = 0 (bandred_tune) */
  int update_lds_cap; /* 1: those launches reserve 20 KB of extra LDS per workgroup (one
                         128 x 128 update workgroup per CU, the rest of the CU left to the
                         panel); 2: never; 0 (default): when the update has at most 8192
                         rows, or the autotuner's choice when b = 0.  Neither knob changes
                         any result bit: every element is still computed by one tile in the
                         same k order */
  int reserved[3];    /* must be zero */
} bandred_opts_t;

/* Symmetric A (n x n) to symmetric band form, bandwidth w, block size b
 * (Sec. 2.1; look-ahead variants of Sec. 2.2).
 *   n    order of A, n >= 0                                      (arg 1)
 *   w    bandwidth, w >= 1                                       (arg 2)
 *   b    block size, 1 <= b <= w (bandred_sy2sb_ex: 0 = tuned, see
 *        bandred_tune)                                           (arg 3)
 *   A    device, lda x n; only the LOWER triangle is read and written; the
 *        strict upper triangle is never referenced                (arg 4)
 *   lda  >= max(1, n)                                            (arg 5)
 *   tau  device, n - w entries when n > w (unused otherwise)      (arg 6)
 * On return B(i,j), 0 <= i-j <= w, holds the band; column c (0 <= c <= n-w-2)
 * holds v[1:] of reflector c in rows c+w+1 .. n-1 (v[0] = 1 at row c+w is
 * implicit) and tau[c] its scalar; tau[n-w-1] = 0.  Q = H_0 H_1 ... and
 * B = Q^T A Q.  When n <= w+1 the matrix is already banded: A is untouched and
 * tau is zero-filled.  Runs on the null stream and returns after completion. */
BANDRED_API int bandred_sy2sb(int64_t n, int64_t w, int64_t b, double *A, int64_t lda,
                  double *tau);

/* General A (m x n, m >= n) to upper triangular-band form, upper bandwidth w,
 * block size b (Sec. 3.1).
 *   m, n  m >= n >= 0                                   (args 1, 2)
 *   w     >= 1; b: 1 <= b <= w                          (args 3, 4)
 *   A     device, lda x n                               (arg 5)
 *   lda   >= max(1, m)                                  (arg 6)
 *   tauq, taup  device, n entries each                  (args 7, 8)
 * On return B(i,j), 0 <= j-i <= w, holds the band.  Left reflector c
 * (c < n) has v[1:] in A(c+1:m-1, c) and scalar tauq[c] (0 when m-c < 2);
 * right reflector c (c <= n-w-2) has u[1:] in A(c, c+w+1:n-1), u[0] = 1 at
 * column c+w, scalar taup[c]; the other taup entries are 0.  U = H_0 H_1 ...,
 * V = G_0 G_1 ..., B = U^T A V.  Null stream, returns after completion. */
BANDRED_API int bandred_ge2gb(int64_t m, int64_t n, int64_t w, int64_t b, double *A,
                  int64_t lda, double *tauq, double *taup);

/* As bandred_sy2sb with a precision form, options and a stream
 * (hipStream_t, NULL = null stream).  Asynchronous: returns once the work is
 * enqueued (argument errors are reported synchronously).  The call may be
 * recorded into a HIP graph (stream capture) once an eager call of the same
 * or a larger size has reserved the workspace; under capture it allocates
 * nothing and returns BANDRED_ERR_UNSUPPORTED otherwise (or while profiling
 * is enabled).  Replays share the device's workspace with every other call:
 * the caller keeps them from overlapping.  A workspace that a captured graph
 * refers to is never freed: when a later eager call needs a larger one, the
 * old one is kept (until the process ends) so that the graph stays valid.
 * Runtime failures are reported by bandred_status.
 * Extra arguments: prec (arg 7), opts (arg 8, may be NULL), stream (arg 9). */
BANDRED_API int bandred_sy2sb_ex(int64_t n, int64_t w, int64_t b, double *A, int64_t lda,
                     double *tau, int prec, const bandred_opts_t *opts,
                     void *stream);

/* As bandred_ge2gb with prec (arg 9), opts (arg 10) and stream (arg 11);
 * asynchronous and capturable like bandred_sy2sb_ex. */
BANDRED_API int bandred_ge2gb_ex(int64_t m, int64_t n, int64_t w, int64_t b, double *A,
                     int64_t lda, double *tauq, double *taup, int prec,
                     const bandred_opts_t *opts, void *stream);

/* General A (m x n, m >= n) to band form with lower AND upper bandwidth w
 * (Sec. 3.3, eqs. updateB0..updateCD22; the left and right updates of the
 * trailing block applied at once, eq. gebrd_2k).  Arguments as
 * bandred_ge2gb_ex: m, n (args 1, 2), w, b (3, 4; 1 <= b <= w), A (5, device,
 * lda x n), lda (6, >= max(1, m)), tauq, taup (7, 8, device, n entries each),
 * prec (9), opts (10, may be NULL), stream (11).
 * On return B(i,j) for -w <= j-i <= w holds the band.  Left reflector c
 * (c <= m-w-2, c < n) has v[0] = 1 implicit at row c+w, v[1:] in
 * A(c+w+1:m-1, c) and scalar tauq[c]; right reflector c (c <= n-w-2) has
 * u[0] = 1 at column c+w, u[1:] in A(c, c+w+1:n-1) and scalar taup[c]; all
 * other tau entries are 0.  U = H_0 H_1 ..., V = G_0 G_1 ..., B = U^T A V.
 * With look-ahead the next left and right panels are factored on a second
 * stream beside the update of the trailing block (Variant V1 when 2b <= w,
 * V2 otherwise).  Asynchronous and capturable like bandred_ge2gb_ex. */
BANDRED_API int bandred_ge2gb_lu(int64_t m, int64_t n, int64_t w, int64_t b, double *A,
                     int64_t lda, double *tauq, double *taup, int prec,
                     const bandred_opts_t *opts, void *stream);

/* Back-transformation: C := Q C (trans = 0) or Q^T C (trans = 1) with the
 * orthogonal factor of bandred_sy2sb, Q = H_0 H_1 ... H_{n-w-1} (Sec. 2.1:
 * the reduction accumulates Q as I + W Y^T panel by panel; eigenvectors of
 * A are Q times those of B).
 *   trans       0 or 1                                              (arg 1)
 *   n, w        as given to the reduction                           (args 2, 3)
 *   b           block of reflectors applied at once, 1 <= b <= 128;
 *               any value gives the same Q                          (arg 4)
 *   A, lda      device, the reduction's output (only the reflectors,
 *               below the band, are read)                           (args 5, 6)
 *   tau         device, n - w entries                               (arg 7)
 *   k           columns of C, >= 0                                  (arg 8)
 *   C, ldc      device, n x k, ldc >= max(1, n), overwritten        (args 9, 10)
 *   stream      hipStream_t or NULL                                 (arg 11)
 * FP64.  Asynchronous; capturable like the _ex calls. */
BANDRED_API int bandred_sy2sb_apply_q(int trans, int64_t n, int64_t w, int64_t b,
                          const double *A, int64_t lda, const double *tau, int64_t k,
                          double *C, int64_t ldc, void *stream);

/* Back-transformation for the general reductions (Sec. 3.1 and 3.3):
 * side 0: C := U C or U^T C (C is m x k); side 1: C := V C or V^T C (C is
 * n x k).  form 0: the factors of bandred_ge2gb (upper triangular-band);
 * form 1: those of bandred_ge2gb_lu (equal bandwidths).  tau is tauq for
 * side 0 and taup for side 1.  Args: side (1), form (2), trans (3), m, n
 * (4, 5), w (6), b (7, 1..128), A (8), lda (9), tau (10), k (11), C (12),
 * ldc (13, >= rows of C), stream (14).  FP64, asynchronous. */
BANDRED_API int bandred_ge2gb_apply(int side, int form, int trans, int64_t m, int64_t n,
                        int64_t w, int64_t b, const double *A, int64_t lda,
                        const double *tau, int64_t k, double *C, int64_t ldc,
                        void *stream);

/* Stage 2 of a two-stage symmetric eigensolver (the paper's pipeline after
 * its first stage, Sec. 4.3): the symmetric band B (bandwidth w) held in the
 * band 0 <= i-j <= w of A (as bandred_sy2sb leaves it) is reduced to a
 * symmetric tridiagonal T = Z^T B Z (Z orthogonal, Z e_0 = e_0) by
 * Householder bulge chasing; on return d (n entries) holds the diagonal of
 * T and e (n-1 entries) its subdiagonal.  T has the eigenvalues of B; its
 * entries are determined by B only up to signs and rounding (two stable
 * tridiagonalisations of one band agree in the spectrum, not entry by
 * entry).  A is only read; Z is not kept.
 *   n (arg 1) >= 0, w (arg 2) >= 1, A (arg 3, device), lda (arg 4 >= n),
 *   d, e (args 5, 6, device), stream (arg 7).
 * Asynchronous; runtime failures (a bounded wait between the sweeps that
 * gave up) are reported by bandred_status. */
BANDRED_API int bandred_sb2st(int64_t n, int64_t w, const double *A, int64_t lda, double *d,
                  double *e, void *stream);

/* All eigenvalues of the symmetric tridiagonal matrix with diagonal d (n
 * entries) and subdiagonal e (n-1 entries), ascending, into lam (n
 * entries); all device pointers.  Multisection (bisection with several
 * points per round) on Sturm counts, accurate to a few units of 2 eps times
 * the Gershgorin bound of |T|.  Args: n (1), d (2),
 * e (3), lam (4), stream (5).  Asynchronous. */
BANDRED_API int bandred_tridiag_eigvals(int64_t n, const double *d, const double *e, double *lam,
                            void *stream);

/* For callers that cannot allocate device memory: code under HIP stream
 * capture with no earlier eager call, serving loops that must not allocate,
 * harnesses that forbid hipMalloc.  Same reduction and arguments as
 * bandred_sy2sb_ex (args 1-7 and stream, arg 8) run in the serial order (no
 * look-ahead stream, no events), with the workspace in a fixed 64 MiB device
 * array that the library holds on each device it runs on until the process
 * ends.  The call allocates nothing: no hipMalloc, hipFree or allocating
 * library routine.  The workspace it needs is about
 * (n - w) * (120 b + b^2 / 8) bytes plus O(b^2 + b w): n <= 3455 at
 * w = b = 128, n <= 8092 at w = b = 64, n <= 16607 at w = b = 32; a larger
 * problem returns BANDRED_ERR_UNSUPPORTED before any work is enqueued (as
 * does a call while profiling is enabled).  BANDRED_INT8_SPLIT_UPDATE needs
 * about 8 (n - w) (n - w + 2 max(2b, w)) bytes more (its digit planes):
 * n <= about 1970 at w = b = 128.  Every call on a device shares
 * that device's array and leaves its contents behind (each call clears what
 * it needs zeroed before use): calls that overlap on one device, on any
 * streams, race and give undefined results; the caller orders them.
 * Asynchronous; runtime failures are reported by bandred_status. */
BANDRED_API int bandred_sy2sb_noalloc(int64_t n, int64_t w, int64_t b, double *A,
                          int64_t lda, double *tau, int prec, void *stream);

/* Many independent symmetric matrices of uneven orders reduced in one
 * persistent launch (not in the paper; same per-matrix result as
 * bandred_sy2sb).
 *   count  number of matrices, >= 0                                  (arg 1)
 *   n      HOST array of count orders                                (arg 2)
 *   w, b   bandwidth and block size for all matrices, 1 <= b <= w    (args 3, 4)
 *   A      HOST array of count DEVICE pointers                       (arg 5)
 *   lda    HOST array of count leading dimensions                    (arg 6)
 *   tau    HOST array of count DEVICE pointers (n[i] - w entries each,
 *          may be NULL for matrices with n[i] <= w)                   (arg 7)
 *   prec   BANDRED_FP64 or BANDRED_FP32_UPDATE                       (arg 8)
 *   stream hipStream_t or NULL                                       (arg 9)
 * Asynchronous like the _ex calls.  The matrix table is uploaded to the
 * device once per distinct content; a call may be captured into a HIP graph
 * after an eager call with the same table.  A table (and the kernel's
 * scratch) that a captured graph refers to is never rewritten or freed by
 * later calls. */
BANDRED_API int bandred_sy2sb_batched(int64_t count, const int64_t *n, int64_t w, int64_t b,
                          double *const *A, const int64_t *lda,
                          double *const *tau, int prec, void *stream);

/* Autotuner (Sec. 4.2: the best block size depends on n and w, and the paper
 * tunes it per problem in steps of 16).  The reduction's result does not
 * depend on b (up to rounding), so b is picked by timing the reduction of a
 * synthetic matrix of the same shape for every candidate b in
 * {16, 32, ..., min(w, 128)} (b = w when w < 16) on the current device; then,
 * at that b, the split between the look-ahead panel and the update beside it
 * (bandred_opts_t.update_chunks in {1, 2, 3, 4} and update_lds_cap in {1, 2},
 * which change no result bit) is picked the same way, and kept when it beats
 * the default by more than 1%.
 *   kind      0: bandred_sy2sb_ex (m ignored), 1: bandred_ge2gb_ex,
 *             2: bandred_ge2gb_lu                                    (arg 1)
 *   m, n, w   problem shape as in those calls                        (args 2-4)
 *   prec      precision form                                         (arg 5)
 *   force     nonzero: measure again even if cached                  (arg 6)
 *   b_out     HOST, receives the chosen b                            (arg 7)
 *   ms_out    HOST, may be NULL: up to cap {b, milliseconds} pairs of the
 *             candidates measured by this call (zeros when it used the
 *             cache)                                                 (args 8, 9)
 * The choice is cached per device in memory and, if the environment variable
 * BANDRED_TUNE_CACHE names a file, appended to it as one JSON object per line
 * ({"kind": ..., "m": ..., "n": ..., "w": ..., "prec": ..., "b": ..., "chunks": ...,
 * "cap": ..., "ms": {...}}), from which later processes read it back.  Synchronous; allocates
 * the trial matrix; must not be called under stream capture.  The _ex calls
 * and bandred_ge2gb_lu accept b = 0 to mean "the tuned b" (tuned on first use
 * outside capture; under capture only a cached choice is used, else
 * BANDRED_ERR_UNSUPPORTED). */
BANDRED_API int bandred_tune(int kind, int64_t m, int64_t n, int64_t w, int prec, int force,
                 int64_t *b_out, double *ms_out, int cap);

/* The autotuner's choice for a problem (kind, m, n, w, prec as for
 * bandred_tune): block size b (arg 6), update_chunks (arg 7) and
 * update_lds_cap (arg 8) as bandred_opts_t defines them (HOST pointers, any
 * may be NULL).  Reads the cache only: returns BANDRED_ERR_UNSUPPORTED when
 * the problem has not been tuned in this process or in the cache file. */
BANDRED_API int bandred_tune_result(int kind, int64_t m, int64_t n, int64_t w, int prec,
                                    int64_t *b, int *update_chunks, int *update_lds_cap);

/* Static description of a status code. */
BANDRED_API const char *bandred_status_string(int status);

/* Runtime status of the asynchronous calls (the _ex and _batched entry
 * points report argument errors at once but run on the device afterwards).
 * Waits for all work on `stream` (hipStream_t, NULL = null stream), then
 * returns the device status word of the most recent call on the current
 * device: 0, or BANDRED_ERR_TIMEOUT when a bounded inter-workgroup wait of a
 * panel factorisation gave up.  In that case the panel kernels of the call
 * exit at their next wait and every later product of the call returns at
 * once, so the outputs are invalid (not partially updated in a defined way).
 * Each call clears the word when it starts: query it after the call whose
 * status is wanted and before the next one on the same device.  Must not be
 * called while `stream` is being captured into a HIP graph. */
BANDRED_API int bandred_status(void *stream);

/* Frees the library's device memory on the current device (workspace,
 * batched tables and scratch, including those kept for captured graphs) after
 * waiting for the device to be idle.  Every HIP graph that captured a call of
 * this library on the device becomes invalid and must not be replayed again.
 * Later calls allocate afresh. */
BANDRED_API int bandred_release(void);

/* Bound of one inter-workgroup wait inside the panel kernels, in
 * microseconds, for later calls on the current device (default 10 s; us <= 0
 * restores the default).  A wait that exceeds it makes the call report
 * BANDRED_ERR_TIMEOUT.  Meant for tests of that error path. */
BANDRED_API int bandred_set_wait_limit_us(double us);

/* Per-kernel-class device time of the most recent call (diagnostics).
 * When enabled (on != 0) every launch is bracketed by HIP events on the
 * stream it runs on; bandred_profile_read fills up to cap entries of
 * {ms, flops, launches} triples (3 doubles per class, classes in the order of
 * bandred_profile_name) and returns the number of classes. */
BANDRED_API int bandred_profile_enable(int on);
BANDRED_API int bandred_profile_read(double *out, int cap);
BANDRED_API const char *bandred_profile_name(int cls);

#ifdef __cplusplus
}
#endif
#endif
