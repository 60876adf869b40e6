// common.hpp -- shared definitions of the gfx950 band-reduction library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/bandred.h"

namespace br {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;   // threads per workgroup for every tiled kernel
constexpr int kNbMax = 128;     // widest panel (block size b) supported
constexpr int kBK = 16;         // k-depth of one LDS stage of the GEMM kernels

// Trailing-update arithmetic (matches bandred_prec_t).
enum Prec { P_F64 = 0, P_F32 = 1, P_SPLIT = 2, P_OZ = 3 };

// exact-split form (ozaki.hip): int8 digits (base 256) per operand entry,
// and the k range after which the int32 accumulators are folded into FP64
constexpr int kOzS = 7;
constexpr int kOzKF = 2048;

// Operand access patterns of the GEMM kernels.
//   A_N:   op(A)(i,k) = A[i + k*lda]
//   A_T:   op(A)(i,k) = A[k + i*lda]
//   A_SYM: op(A)(i,k) = A[max(i,k) + min(i,k)*lda]  (symmetric, lower stored)
//   B_N:   op(B)(k,j) = B[k + j*ldb]
//   B_T:   op(B)(k,j) = B[j + k*ldb]
//   B_TROT:op(B)(k,j) = B[j + ((k + rot) mod K)*ldb]
enum OpA { A_N = 0, A_T = 1, A_SYM = 2 };
enum OpB { B_N = 0, B_T = 1, B_TROT = 2 };

// Epilogues.
//   E_AXPBY:  C = alpha*acc + beta*C  (C not read when beta == 0)
//   E_PART:   part[z] = acc           (split-K partial, column-major ld M)
//   E_SYR2K:  C -= acc on the lower triangle (row >= col) of a column range
enum Epi { E_AXPBY = 0, E_PART = 1, E_SYR2K = 2 };

struct GemmDesc {
  int M, N, K;
  const double *A;
  int64_t lda;
  const double *B;
  int64_t ldb;
  double *C;
  int64_t ldc;
  double alpha, beta;
  int kchunk;      // k-range handled by one blockIdx.z (multiple of kBK)
  double *part;    // E_PART output: part + z*M*N, column-major ld M
  int rot;         // B_TROT rotation
  int c0, c1;      // E_SYR2K: columns [c0, c1) of C, rows >= c0
  const int *gate; // when set, the kernel runs only if *gate == gate_val
  int gate_val;
  int tile64;      // nonzero: 64 x 64 output tiles (4x the workgroups of 128 x 128)
  double *C2;      // E_AXPBY: when set, every stored value also goes to C2 ...
  int64_t ldc2;
  int c2_trans;    // ... at (row, col) (ld ldc2), or transposed at (col, row)
  int prio;        // nonzero: the waves run at raised issue priority (panel products)
  int lds_pad;     // extra LDS bytes reserved per workgroup (limits residency per CU)
  const int *abort;// when set and nonzero at launch, the kernel returns at once (a
                   // panel factorisation of the same call gave up a bounded wait)
};

// Wave issue priority of the panel kernels.  The panel of the next step runs
// beside the trailing update (look-ahead) and is the longer of the two; at a
// raised priority its waves are issued ahead of the update's waves on a
// shared SIMD.  kPrioCrit is for the one wave on the Cholesky / LU pivot chain.
constexpr int kPrioPanel = 2;
constexpr int kPrioCrit = 3;

struct PanelDesc {
  double *P;        // panel, element (r,k) at P[r*rs + k*cs]
  int64_t ldp;      // the stride that is not 1
  int m, nb, R;     // rows, columns, rows per workgroup
  double *V;        // explicit V (m x nb, column-major, unit diagonal, zero above)
  int64_t ldv;
  double *tau;      // nb scalars
  double *part;     // [2][gridDim.x][kNbMax] partial dot products
  double *piv;      // [kNbMax][kNbMax] pivot rows
  unsigned *counter;// arrival counter, zero at launch
  int *status;      // set to 4 (timeout) if a wait gives up
  int *abort_flag;  // raised by the first workgroup that gives up
  long long timeout_ticks;  // bound of one wait, in s_memrealtime ticks
  const int *gate;  // when set, the kernel runs only if *gate == gate_val
  int gate_val;
};

}  // namespace br

#define BR_HIP_CHECK(expr)                                  \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return br::hip_fail(_e, #expr);   \
  } while (0)

namespace br {
int hip_fail(hipError_t e, const char *what);

// host-side launchers (defined in gemm.hip / panel.hip)
int launch_gemm(int opa, int opb, int epi, int prec, const GemmDesc &d, int ksplit,
                hipStream_t s);
// output tile of launch_gemm for an M x N product (tile64: force 64 x 64)
int gemm_tile_shape(int epi, int M, int N, int tile64, int *tm, int *tn);
int launch_reduce_partials(const double *part, int ksplit, int M, int N, double alpha,
                           double *C, int64_t ldc, double beta, hipStream_t s,
                           const int *gate = nullptr, int gate_val = 0,
                           const int *abort = nullptr);
int launch_panel(bool rowmajor, const PanelDesc &d, int nwg, hipStream_t s);
int launch_larft(const double *S, int ldS, const double *tau, int nb, double *T, int ldT,
                 hipStream_t s, const int *gate = nullptr, int gate_val = 0);
int launch_chol_inv(const double *G, int ldg, int b, double rel, double *R, double *Rinv, int *flag,
                    const int *structure, hipStream_t s);
int launch_recon(const double *Qtop, int ldq, int b, double *V, int64_t ldv, double *T, int ldt,
                 double *tau, double *Uinv, double *sgn, double *Uscr, const int *flag,
                 hipStream_t s);
int launch_panel_structure(const double *P, int64_t ldp, int rowmajor, int m, int b,
                           int *structure, hipStream_t s);
int launch_panel_finalize(double *P, int64_t ldp, int rowmajor, int m, int b, const double *V,
                          int64_t ldv, const double *Rh0, const double *sgn, const int *flag,
                          hipStream_t s);
int launch_extract_v(const double *A, int64_t lda, int rowstore, int64_t r0, int64_t i0, int pb,
                     int j, double *V, int64_t ldv, hipStream_t s);
// block size picked by the autotuner (tune.hip) for a call with b = 0
// (kind 0: sy2sb, 1: ge2gb, 2: ge2gb_lu)
int tune_pick(int kind, int64_t m, int64_t n, int64_t w, int prec, hipStream_t s, int *b_out,
              int *chunks, int *cap);
int tune_lookup(int kind, int64_t m, int64_t n, int64_t w, int prec);
// stage 2 (stage2.hip): band -> tridiagonal by bulge chasing, tridiagonal eigenvalues
int launch_sb2st(const double *A, int64_t lda, int n, int w, double *AB, int64_t ldab,
                 unsigned *sweep_ctr, int *progress, int *flags, long long timeout_ticks, int nwg,
                 double *dg, double *e, hipStream_t s);
int launch_tridiag_eig(const double *dg, const double *e, int n, double *bounds, double *lam,
                       hipStream_t s);
// exact-split products (ozaki.hip).  The inner dimension K is one segment,
// or two ([0, ks) and [ks, K)) with scales of their own; the digit planes
// hold each segment padded to a multiple of 64 (oz_plane_cols: total columns,
// *L0 = where segment 1 starts).
int oz_plane_cols(int K, int ks, int *L0);
// op(A) (isB = 0) or op(B) (isB = 1) as rows of kOzS int8 digit planes
// (rows x Kp each) with exponents ex[seg rows + r]; rmax is scratch of
// 2 rows words of 64 bits
// (rmax_in: the row maxima already known, as the bits of the doubles -- one
// segment; the pass that finds them is skipped)
int oz_slice(const double *X, int64_t ld, int op, int rows, int K, int ks, int rot, int isB,
             unsigned long long *rmax, int *ex, int8_t *planes, hipStream_t s,
             const unsigned long long *rmax_in = nullptr);
// (rec, SYR2K only: atomicMax of the result's row and column maxima for
// indices >= rec_off into rec[index - rec_off])
int oz_gemm(int epi, const int8_t *PA, const int8_t *PB, const int *ea, const int *eb, int M,
            int N, int Kp, int L0, int ksplit, int kchunk, double *C, int64_t ldc, double alpha,
            double beta, double *part, int c0, int c1, const int *abort, hipStream_t s,
            unsigned long long *rec = nullptr, int rec_off = 0);
constexpr int kPackedMax = kNbMax * (kNbMax + 1) / 2;
int launch_fill(double *p, int64_t count, double v, hipStream_t s);
int launch_fill_u32(unsigned *p, int64_t count, unsigned v, hipStream_t s);
int panel_lds_bytes(int R, int nb);

// One matrix of a batched SY2SB call (device table entry).
struct BatchEntry {
  double *A;
  double *tau;
  int64_t lda;
  int n;
  int pad;
};
int launch_batched(int prec, const BatchEntry *table, int count, int w, int b, unsigned *queue,
                   double *ws, int nwg, hipStream_t s);
int64_t batched_ws_doubles();   // scratch doubles per workgroup
int batched_max_trailing();     // largest n - w the batched kernel holds
int batched_max_block();        // largest b of the batched kernel
}  // namespace br
