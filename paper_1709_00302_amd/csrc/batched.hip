// batched.hip -- many independent SY2SB reductions in one persistent launch
// (gfx950).  Not in the paper: its blocked algorithm (Sec. 2.1, eqs.
// updateA0 to updateA2syr2k) applied to thousands of small matrices.
//
// One workgroup (8 waves) reduces one whole matrix at a time; workgroups take
// matrices from an atomic counter over a table sorted by decreasing order
// (largest first), so the launch needs no host synchronisation and balances
// uneven sizes.  Per panel of pb <= 16 columns (r = c + w, j = n - r):
//   1. Householder QR of the j x pb panel held in registers (2 rows per
//      thread), one workgroup reduction per column;
//   2. S = V^T V, T by the compact-WY recurrence, Wt = V T;
//   3. A1 -= V (Wt^T A1) on the w - pb in-band columns (pb < w only);
//   4. X = A2 Wt: every lower 16 x 16 block A_IK of A2 is read once and used
//      twice, X_I += A_IK Wt_K and X_K += A_IK^T Wt_I (transposed through a
//      per-wave LDS tile); X accumulates in LDS;
//   5. M = Wt^T X, W = X - 1/2 V M;
//   6. A2 -= W V^T + V W^T on the lower blocks.
// When w = b = 16 the next panel is the first column block of A2 and the
// block grids of consecutive trailing matrices coincide, so steps 6 and 4 of
// consecutive panels are fused (the paper's look-ahead, Sec. 2.2, inside one
// workgroup): after step 5 the first column block of A2 is updated, the next
// panel is factored (1, 2), and a single pass over the remaining lower blocks
// applies this panel's update to each block and, from the updated block in
// registers, accumulates the next panel's X.  Every lower block is then read
// and written once per panel.
//
// Products run on 16 x 16 x 4 MFMA blocks: FP64, or FP32 for the trailing
// products 4 and 6 in the FP32-update form.  V and W live in a per-workgroup
// scratch column-major and Wt row-major, rows padded to a multiple of 16, so
// that every operand fragment of the O(j^2) passes is read with 16
// consecutive lanes on 16 consecutive doubles.  In those passes each wave
// owns whole column blocks (dealt in snake order) and loads the next block's
// operands before it uses the current ones.
#include "common.hpp"

namespace br {

constexpr int kBT = 512;              // threads per workgroup (8 waves)
constexpr int kBW = kBT / 64;         // waves
constexpr int kBN = 16;               // panel width of the batched path
constexpr int kRPT = 2;               // panel rows per thread
constexpr int kBJMax = kBT * kRPT;    // largest trailing order j = n - w
constexpr int64_t kPanelD = (int64_t)kBJMax * kBN;  // doubles of one scratch panel
constexpr int kTS = kBN + 1;          // row stride of the transpose tiles (bank spread)

struct BatchDesc {
  const BatchEntry *table;
  int count;
  int w, b;
  unsigned *queue;
  double *ws;          // per-workgroup scratch: V[2], W, Wt, each kBJMax x 16
  int64_t ws_stride;   // doubles per workgroup
};

// The matrices' addresses come from the device table, so the compiler cannot
// tell that they are global memory; these accessors say so (global rather
// than flat instructions, which the wait counters track more precisely).
// Offsets are 32-bit element counts below 2^29 (checked by the host), so
// the byte offset fits the 32-bit offset register of a global access with a
// uniform base.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ double gld(const double *p, uint32_t i) {
  return *(const gdouble *)((const gchar *)p + (i << 3));
}
__device__ __forceinline__ void gst(double *p, uint32_t i, double v) {
  *(gdouble *)((gchar *)p + (i << 3)) = v;
}

template <int PREC>
__device__ __forceinline__ int orow(int lane, int e) {
  return (PREC == P_F64) ? (lane >> 4) + 4 * e : 4 * (lane >> 4) + e;
}

// acc += A B for 16 x 16 blocks with inner dimension 16;
// a[s] = A(l%16, k_s(l)), b[s] = B(k_s(l), l%16) for any bijection k_s(l)
// of the 16 inner indices shared by both operands (l = lane).
template <int PREC>
__device__ __forceinline__ void mma16(v4d &acc64, v4f &acc32, const double *a, const double *b) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if constexpr (PREC == P_F64)
      acc64 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc64, 0, 0, 0);
    else
      acc32 = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a[s], (float)b[s], acc32, 0, 0, 0);
  }
}

template <int PREC>
__device__ __forceinline__ double accv(const v4d &a64, const v4f &a32, int e) {
  return (PREC == P_F64) ? a64[e] : (double)a32[e];
}

// ---- cross-lane moves of doubles (VALU only) --------------------------------
__device__ __forceinline__ int lo32(double x) { return (int)(__double_as_longlong(x) & 0xffffffffLL); }
__device__ __forceinline__ int hi32(double x) { return (int)(__double_as_longlong(x) >> 32); }
__device__ __forceinline__ double mk64(int lo, int hi) {
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ double dpp64(double x) {
  return mk64(__builtin_amdgcn_update_dpp(0, lo32(x), CTRL, 0xf, 0xf, false),
              __builtin_amdgcn_update_dpp(0, hi32(x), CTRL, 0xf, 0xf, false));
}
// x + y after swapping lanes 32..63 of x with lanes 0..31 of y: lanes 0..31
// get x(l) + x(l+32), lanes 32..63 get y(l-32) + y(l)
__device__ __forceinline__ double swapsum32(double x, double y) {
  auto l = __builtin_amdgcn_permlane32_swap((unsigned)lo32(x), (unsigned)lo32(y), false, false);
  auto h = __builtin_amdgcn_permlane32_swap((unsigned)hi32(x), (unsigned)hi32(y), false, false);
  return mk64((int)l[0], (int)h[0]) + mk64((int)l[1], (int)h[1]);
}
// the same across the 16-lane rows: odd rows of x with even rows of y
__device__ __forceinline__ double swapsum16(double x, double y) {
  auto l = __builtin_amdgcn_permlane16_swap((unsigned)lo32(x), (unsigned)lo32(y), false, false);
  auto h = __builtin_amdgcn_permlane16_swap((unsigned)hi32(x), (unsigned)hi32(y), false, false);
  return mk64((int)l[0], (int)h[0]) + mk64((int)l[1], (int)h[1]);
}
constexpr int kDppRowMirror = 0x140;      // lane i <-> 15 - i within 16
constexpr int kDppHalfMirror = 0x141;     // lane i <-> 7 - i within 8
constexpr int kDppQuadSwap2 = 0x4e;       // quad_perm [2,3,0,1]
constexpr int kDppQuadSwap1 = 0xb1;       // quad_perm [1,0,3,2]

// Sum of 16 per-lane values over the wave by recursive halving: at each level
// a lane keeps half of its values and adds the partner's copy of that half
// (partners differ in lane bit 5, 4, 3, 2; then 1 and 0 sum the last value).
// On return lane l holds the total of value sum16_index(l).
__device__ __forceinline__ double wave_sum16(const double (&v)[kBN], int lane) {
  const bool b3 = lane & 8, b2 = lane & 4;
  double h8[8], h4[4], h2[2];
#pragma unroll
  for (int t = 0; t < 8; ++t) h8[t] = swapsum32(v[t], v[8 + t]);
#pragma unroll
  for (int t = 0; t < 4; ++t) h4[t] = swapsum16(h8[t], h8[4 + t]);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const double keep = b3 ? h4[2 + t] : h4[t], send = b3 ? h4[t] : h4[2 + t];
    h2[t] = keep + dpp64<kDppRowMirror>(send);
  }
  const double keep = b2 ? h2[1] : h2[0], send = b2 ? h2[0] : h2[1];
  double h1 = keep + dpp64<kDppHalfMirror>(send);
  h1 += dpp64<kDppQuadSwap2>(h1);
  h1 += dpp64<kDppQuadSwap1>(h1);
  return h1;
}

__device__ __forceinline__ int sum16_index(int lane) {
  return ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
}

__device__ __forceinline__ double readlane64(double x, int l) {
  return mk64(__builtin_amdgcn_readlane(lo32(x), l), __builtin_amdgcn_readlane(hi32(x), l));
}

struct BatchLds {
  double X[kBJMax * kBN];        // X accumulator, row-major j x 16
  double scr[kBW][kBN * kTS];    // per-wave partial products / transpose tiles
  double S[kBN * kBN], T[kBN * kBN], M[kBN * kBN];
  double red[2][kBW][kBN];       // per-wave column sums (double buffered)
  double prow[2][kBN];           // pivot row (double buffered)
  double tau[kBN];
  int item;
};

// Sum the 8 waves' 16 x 16 FP64 partial blocks into dst (row-major, LDS).
__device__ __forceinline__ void reduce_waves(BatchLds &L, const v4d &acc, double *dst, int tid,
                                             int lane, int wave) {
#pragma unroll
  for (int e = 0; e < 4; ++e) L.scr[wave][orow<P_F64>(lane, e) * kBN + (lane & 15)] = acc[e];
  __syncthreads();
  if (tid < kBN * kBN) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kBW; ++q) s += L.scr[q][tid];
    dst[tid] = s;
  }
  __syncthreads();
}

// Column I of the panel QR (I fixed at compile time so that the register
// panel a[][] is never indexed dynamically).  One workgroup barrier per
// column: each wave reduces its sums s_k = sum_{rho > I} a(rho, I) a(rho, k)
// to LDS, and after the barrier every wave adds up the eight partial sums
// itself (lane l for column l % 16) and broadcasts them with readlane.
template <int I>
__device__ __forceinline__ void house_col(double (&a)[kRPT][kBN], BatchLds &L, int tid, int lane,
                                          int wave, int pb, double *tau_out) {
  if (I >= pb) return;
  constexpr int buf = I & 1;
  double part[kBN];
#pragma unroll
  for (int k = 0; k < kBN; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < kRPT; ++s)
      if (s > 0 || tid > I) acc += a[s][I] * a[s][k];
    part[k] = acc;
  }
  const double q = wave_sum16(part, lane);
  if ((lane & 3) == 0) L.red[buf][wave][sum16_index(lane)] = q;
  if (tid == I) {
#pragma unroll
    for (int k = 0; k < kBN; ++k) L.prow[buf][k] = a[0][k];
  }
  __syncthreads();
  // lane l: column l % 16, waves l / 16 and l / 16 + 4, then over the 4 rows
  const int kc = lane & 15;
  double t = L.red[buf][lane >> 4][kc] + L.red[buf][(lane >> 4) + 4][kc];
  t = swapsum16(t, t);  // rows 0+1 and 2+3 (each lane gets its pair's sum)
  t = swapsum32(t, t);  // halves
  const double pk = L.prow[buf][kc];
  // reflector: beta = -sign(alpha) ||(alpha, x)||, v = x / (alpha - beta)
  const double alpha = readlane64(pk, I), sig2 = readlane64(t, I);
  double tau = 0.0, dv = 0.0, beta = alpha;
  if (sig2 != 0.0) {
    const double nrm = sqrt(alpha * alpha + sig2);
    beta = (alpha < 0.0) ? nrm : -nrm;
    tau = (beta - alpha) / beta;
    dv = 1.0 / (alpha - beta);
  }
  if (tau != 0.0) {
    // column k: a_k -= tau v (v^T a_k) with v^T a_k = p_k + s_k / (alpha - beta)
    const double fl = tau * (pk + t * dv);
    double f[kBN];
#pragma unroll
    for (int k = I + 1; k < kBN; ++k) f[k] = readlane64(fl, k);
#pragma unroll
    for (int s = 0; s < kRPT; ++s) {
      if (s > 0 || tid > I) {
        const double v = a[s][I] * dv;
        a[s][I] = v;
#pragma unroll
        for (int k = I + 1; k < kBN; ++k) a[s][k] -= v * f[k];
      }
    }
    if (tid == I) {
#pragma unroll
      for (int k = I + 1; k < kBN; ++k) a[0][k] -= f[k];
    }
  }
  if (tid == I) a[0][I] = beta;
  if (tid == 0) {
    L.tau[I] = tau;
    gst(tau_out, I, tau);
  }
}

template <int I>
struct ColLoop {
  static __device__ __forceinline__ void run(double (&a)[kRPT][kBN], BatchLds &L, int tid, int lane,
                                             int wave, int pb, double *tau_out) {
    house_col<I>(a, L, tid, lane, wave, pb, tau_out);
    ColLoop<I + 1>::run(a, L, tid, lane, wave, pb, tau_out);
  }
};
template <>
struct ColLoop<kBN> {
  static __device__ __forceinline__ void run(double (&)[kRPT][kBN], BatchLds &, int, int, int, int,
                                             double *) {}
};

struct Lane {
  int tid, lane, wave, l16, l4;
};

// Column block K of the snake order: round r deals blocks r*8 .. r*8+7 to the
// waves, reversed on odd rounds.
__device__ __forceinline__ int snake(int kk) {
  const int round = kk / kBW, pos = kk % kBW;
  return round * kBW + ((round & 1) ? kBW - 1 - pos : pos);
}

// 1 + 2: QR of the j x pb panel P (in place, tau to tau_out), explicit V
// (column-major, unit diagonal, zero padding), S, T and Wt = V T.
__device__ __forceinline__ void factor_panel(BatchLds &L, const Lane &q, double *P, int lda,
                                             int j, int pb, double *tau_out, double *Vc,
                                             double *Wt) {
  const int nbk = (j + kBN - 1) / kBN;
  const v4d z64 = {0.0, 0.0, 0.0, 0.0};
  const v4f z32 = {0.0f, 0.0f, 0.0f, 0.0f};
  double a[kRPT][kBN];
#pragma unroll
  for (int s = 0; s < kRPT; ++s) {
    const int rho = q.tid + kBT * s;
#pragma unroll
    for (int k = 0; k < kBN; ++k) {
      const double v = gld(P, min(rho, j - 1) + min(k, pb - 1) * lda);
      a[s][k] = (rho < j && k < pb) ? v : 0.0;
    }
  }
  ColLoop<0>::run(a, L, q.tid, q.lane, q.wave, pb, tau_out);
#pragma unroll
  for (int s = 0; s < kRPT; ++s) {
    const int rho = q.tid + kBT * s;
    if (rho < j) {
#pragma unroll
      for (int k = 0; k < kBN; ++k)
        if (k < pb) gst(P, rho + k * lda, a[s][k]);
    }
    if (rho < nbk * kBN) {
#pragma unroll
      for (int k = 0; k < kBN; ++k) {
        double v = 0.0;
        if (k < pb && rho < j) v = (rho == k) ? 1.0 : (rho > k ? a[s][k] : 0.0);
        gst(Vc, k * kBJMax + rho, v);
      }
    }
  }
  __syncthreads();
  {
    v4d acc = z64;
    v4f acc32 = z32;
    for (int I = q.wave; I < nbk; I += kBW) {
      double av[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) av[s] = gld(Vc, q.l16 * kBJMax + I * kBN + q.l4 + 4 * s);
      mma16<P_F64>(acc, acc32, av, av);  // V^T(l%16, k) and V(k, l%16) are the same value
    }
    reduce_waves(L, acc, L.S, q.tid, q.lane, q.wave);
  }
  if (q.wave == 0) {
    // T(i,i) = tau_i, T(0:i, i) = -tau_i T(0:i, 0:i) S(0:i, i); lane l
    // holds row l of T
    double trow[kBN];
#pragma unroll
    for (int i = 0; i < kBN; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < i; ++m) acc += trow[m] * L.S[m * kBN + i];
      const double ti = (i < pb) ? L.tau[i] : 0.0;
      trow[i] = (q.lane < i) ? -ti * acc : (q.lane == i ? ti : 0.0);
    }
    if (q.lane < kBN) {
#pragma unroll
      for (int i = 0; i < kBN; ++i) L.T[q.lane * kBN + i] = trow[i];
    }
  }
  __syncthreads();
  for (int I = q.wave; I < nbk; I += kBW) {
    v4d acc = z64;
    v4f acc32 = z32;
    double av[4], bv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      av[s] = gld(Vc, (q.l4 + 4 * s) * kBJMax + I * kBN + q.l16);
      bv[s] = L.T[(q.l4 + 4 * s) * kBN + q.l16];
    }
    mma16<P_F64>(acc, acc32, av, bv);
#pragma unroll
    for (int e = 0; e < 4; ++e)
      gst(Wt, (I * kBN + orow<P_F64>(q.lane, e)) * kBN + q.l16, acc[e]);
  }
  __syncthreads();
}

// 3: A1 (j x a1w, columns right of the panel inside the band) -= V (Wt^T A1).
__device__ __forceinline__ void update_a1(BatchLds &L, const Lane &q, double *A1, int lda,
                                          int j, int a1w, const double *Vc, const double *Wt) {
  const int nbk = (j + kBN - 1) / kBN;
  const v4d z64 = {0.0, 0.0, 0.0, 0.0};
  const v4f z32 = {0.0f, 0.0f, 0.0f, 0.0f};
  const int nq = (a1w + kBN - 1) / kBN;
  for (int Q = 0; Q < nq; ++Q) {
    v4d acc = z64;
    v4f acc32 = z32;
    for (int I = q.wave; I < nbk; I += kBW) {
      double av[4], bv[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = I * kBN + q.l4 + 4 * s, col = Q * kBN + q.l16;
        av[s] = gld(Wt, row * kBN + q.l16);
        bv[s] = (row < j && col < a1w) ? gld(A1, row + col * lda) : 0.0;
      }
      mma16<P_F64>(acc, acc32, av, bv);
    }
    reduce_waves(L, acc, L.M, q.tid, q.lane, q.wave);  // Z_Q, kept in the M buffer
    for (int I = q.wave; I < nbk; I += kBW) {
      // D(a, c) = sum_k Z(k, a) V_I(c, k) = (V_I Z)(c, a): lanes run down rows of A1
      v4d o = z64;
      v4f o32 = z32;
      double av[4], bv[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        av[s] = L.M[(q.l4 + 4 * s) * kBN + q.l16];
        bv[s] = gld(Vc, (q.l4 + 4 * s) * kBJMax + I * kBN + q.l16);
      }
      mma16<P_F64>(o, o32, av, bv);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = I * kBN + q.l16, col = Q * kBN + orow<P_F64>(q.lane, e);
        if (row < j && col < a1w) gst(A1, row + col * lda, gld(A1, row + col * lda) - o[e]);
      }
    }
    __syncthreads();
  }
}

// The O(j^2) passes below walk the row blocks I of a wave-owned column block
// with the operands of blocks I+1 (and I+2) already requested.  The loops
// are unrolled by the pipeline depth so that each stage keeps its registers
// (a register copy of a pending load would wait for it), and loads past the
// last block reload the last block instead of branching (harmless, and it
// keeps the wait counters exact).

// 4: X = A2 Wt from the lower blocks of A2 (read only).
template <int PREC>
__device__ __forceinline__ void x_pass(BatchLds &L, const Lane &q, const double *A2, int lda,
                                       int j, const double *Wt) {
  const int nbk = (j + kBN - 1) / kBN;
  const v4d z64 = {0.0, 0.0, 0.0, 0.0};
  const v4f z32 = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int t = q.tid; t < nbk * kBN * kBN; t += kBT) L.X[t] = 0.0;
  __syncthreads();
  double *tile = L.scr[q.wave];
  struct Stage {
    double a[4], t[4];
  };
  for (int kk = q.wave; kk < nbk + kBW; kk += kBW) {
    const int K = snake(kk);
    if (K >= nbk) continue;
    v4d xk = z64;
    v4f xk32 = z32;
    double wtk[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) wtk[s] = gld(Wt, (K * kBN + q.l4 + 4 * s) * kBN + q.l16);
    // lane l holds A_IK(l%16, l/16 + 4s) (the diagonal block mirrored), masked where used
    auto load = [&](int I, Stage &S) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = I * kBN + q.l16, col = K * kBN + q.l4 + 4 * s;
        const int rr = min(max(row, col), j - 1), cc = min(min(row, col), j - 1);
        S.a[s] = gld(A2, rr + cc * lda);
        S.t[s] = gld(Wt, (I * kBN + q.l4 + 4 * s) * kBN + q.l16);
      }
    };
    auto body = [&](int I, const Stage &S) {
      double ak[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = I * kBN + q.l16, col = K * kBN + q.l4 + 4 * s;
        ak[s] = (row < j && col < j) ? S.a[s] : 0.0;
      }
      v4d o = z64;
      v4f o32 = z32;
      mma16<PREC>(o, o32, ak, wtk);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        atomicAdd(&L.X[(I * kBN + orow<PREC>(q.lane, e)) * kBN + q.l16], accv<PREC>(o, o32, e));
      if (I > K) {
#pragma unroll
        for (int s = 0; s < 4; ++s) tile[(q.l4 + 4 * s) * kTS + q.l16] = ak[s];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double at[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) at[s] = tile[q.l16 * kTS + q.l4 + 4 * s];  // A_IK(l/16 + 4s, l%16)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        mma16<PREC>(xk, xk32, at, S.t);
      }
    };
    Stage S0, S1;
    load(K, S0);
    for (int I = K; I < nbk; I += 2) {
      load(min(I + 1, nbk - 1), S1);
      body(I, S0);
      if (I + 1 >= nbk) break;
      load(min(I + 2, nbk - 1), S0);
      body(I + 1, S1);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      atomicAdd(&L.X[(K * kBN + orow<PREC>(q.lane, e)) * kBN + q.l16], accv<PREC>(xk, xk32, e));
  }
  __syncthreads();
}

// 5: M = Wt^T X; W = X - 1/2 V M (stored column-major).
__device__ __forceinline__ void form_w(BatchLds &L, const Lane &q, int j, const double *Vc,
                                       const double *Wt, double *Wc) {
  const int nbk = (j + kBN - 1) / kBN;
  const v4d z64 = {0.0, 0.0, 0.0, 0.0};
  const v4f z32 = {0.0f, 0.0f, 0.0f, 0.0f};
  {
    v4d acc = z64;
    v4f acc32 = z32;
    for (int I = q.wave; I < nbk; I += kBW) {
      double av[4], bv[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = I * kBN + q.l4 + 4 * s;
        av[s] = gld(Wt, row * kBN + q.l16);
        bv[s] = L.X[row * kBN + q.l16];
      }
      mma16<P_F64>(acc, acc32, av, bv);
    }
    reduce_waves(L, acc, L.M, q.tid, q.lane, q.wave);
  }
  for (int I = q.wave; I < nbk; I += kBW) {
    v4d o = z64;
    v4f o32 = z32;
    double av[4], bv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      av[s] = gld(Vc, (q.l4 + 4 * s) * kBJMax + I * kBN + q.l16);
      bv[s] = L.M[(q.l4 + 4 * s) * kBN + q.l16];
    }
    mma16<P_F64>(o, o32, av, bv);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = I * kBN + orow<P_F64>(q.lane, e);
      gst(Wc, q.l16 * kBJMax + row, L.X[row * kBN + q.l16] - 0.5 * o[e]);
    }
  }
  __syncthreads();
}

// Operands of the rank-2b update of block (I, K): A operands V_K(a, k),
// W_K(a, k) (a = l%16, k = l/16 + 4s) are loaded per column; B operands
// W_I(c, k), V_I(c, k) (c = l%16) per block.  The update
//   D(a, c) = sum_k V_K(a, k) W_I(c, k) + W_K(a, k) V_I(c, k)
// is element (I*16 + c, K*16 + a) of W V^T + V W^T, so lane l owns rows
// I*16 + l%16 and columns K*16 + orow(l, e) of the block.
__device__ __forceinline__ void load_vw(const double *Vc, const double *Wc, int B, int l16, int l4,
                                        double (&vb)[4], double (&wb)[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    vb[s] = gld(Vc, (l4 + 4 * s) * kBJMax + B * kBN + l16);
    wb[s] = gld(Wc, (l4 + 4 * s) * kBJMax + B * kBN + l16);
  }
}

struct UpdStage {
  double w[4], v[4], a[4], t[4];
};

// Operands of block (I, K) of the update (and, with Wtn, of the next X):
// W_I, V_I, the block of A2 (lane: rows I*16 + l%16, columns K*16 + orow),
// and Wt'_{I-1} with inner index orow.
template <int PREC, bool NEXT>
__device__ __forceinline__ void load_upd(const Lane &q, const double *A2, int lda, int j,
                                         const double *Vc, const double *Wc, const double *Wtn,
                                         int I, int K, UpdStage &S) {
  load_vw(Vc, Wc, I, q.l16, q.l4, S.v, S.w);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int row = I * kBN + q.l16, col = K * kBN + orow<PREC>(q.lane, e);
    const int cc = min(col, j - 1), rr = min(max(row, cc), j - 1);
    S.a[e] = gld(A2, rr + cc * lda);  // masked where used
    if constexpr (NEXT) S.t[e] = gld(Wtn, ((I - 1) * kBN + orow<PREC>(q.lane, e)) * kBN + q.l16);
  }
}

// A_IK - (W V^T + V W^T)_IK of one block; stored on the lower triangle.
// Returns the new block values (zero outside the stored part) in an[].
template <int PREC>
__device__ __forceinline__ void upd_block(const Lane &q, double *A2, int lda, int j, int I,
                                          int K, const double (&vk)[4], const double (&wk)[4],
                                          const UpdStage &S, double (&an)[4]) {
  const v4d z64 = {0.0, 0.0, 0.0, 0.0};
  const v4f z32 = {0.0f, 0.0f, 0.0f, 0.0f};
  v4d o = z64, o2 = z64;
  v4f o32 = z32, o232 = z32;
  mma16<PREC>(o, o32, vk, S.w);
  mma16<PREC>(o2, o232, wk, S.v);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int row = I * kBN + q.l16, col = K * kBN + orow<PREC>(q.lane, e);
    const bool ok = row < j && row >= col;
    an[e] = ok ? S.a[e] - (accv<PREC>(o, o32, e) + accv<PREC>(o2, o232, e)) : 0.0;
    if (ok) gst(A2, row + col * lda, an[e]);
  }
}

// 6: A2 -= W V^T + V W^T on the lower blocks.
template <int PREC>
__device__ __forceinline__ void syr2k_pass(const Lane &q, double *A2, int lda, int j,
                                           const double *Vc, const double *Wc) {
  const int nbk = (j + kBN - 1) / kBN;
  for (int kk = q.wave; kk < nbk + kBW; kk += kBW) {
    const int K = snake(kk);
    if (K >= nbk) continue;
    double vk[4], wk[4], an[4];
    load_vw(Vc, Wc, K, q.l16, q.l4, vk, wk);
    UpdStage S0, S1;
    load_upd<PREC, false>(q, A2, lda, j, Vc, Wc, nullptr, K, K, S0);
    for (int I = K; I < nbk; I += 2) {
      load_upd<PREC, false>(q, A2, lda, j, Vc, Wc, nullptr, min(I + 1, nbk - 1), K, S1);
      upd_block<PREC>(q, A2, lda, j, I, K, vk, wk, S0, an);
      if (I + 1 >= nbk) break;
      load_upd<PREC, false>(q, A2, lda, j, Vc, Wc, nullptr, min(I + 2, nbk - 1), K, S0);
      upd_block<PREC>(q, A2, lda, j, I + 1, K, vk, wk, S1, an);
    }
  }
  __syncthreads();
}

// Look-ahead: the rank-2b update of the first column block of A2 only (the
// band's diagonal block and the next panel).
template <int PREC>
__device__ __forceinline__ void syr2k_col0(const Lane &q, double *A2, int lda, int j,
                                           const double *Vc, const double *Wc) {
  const int nbk = (j + kBN - 1) / kBN;
  double vk[4], wk[4], an[4];
  load_vw(Vc, Wc, 0, q.l16, q.l4, vk, wk);
  UpdStage S0, S1;
  load_upd<PREC, false>(q, A2, lda, j, Vc, Wc, nullptr, min(q.wave, nbk - 1), 0, S0);
  for (int I = q.wave; I < nbk; I += 2 * kBW) {
    load_upd<PREC, false>(q, A2, lda, j, Vc, Wc, nullptr, min(I + kBW, nbk - 1), 0, S1);
    upd_block<PREC>(q, A2, lda, j, I, 0, vk, wk, S0, an);
    if (I + kBW >= nbk) break;
    load_upd<PREC, false>(q, A2, lda, j, Vc, Wc, nullptr, min(I + 2 * kBW, nbk - 1), 0, S0);
    upd_block<PREC>(q, A2, lda, j, I + kBW, 0, vk, wk, S1, an);
  }
  __syncthreads();
}

// Fused 6 + 4: for the lower blocks (I, K), K >= 1, of A2: A_IK -= (W V^T +
// V W^T)_IK with this panel's V, W; then, with the updated block, X'_{I-1} +=
// A_IK Wt'_{K-1} and X'_{K-1} += A_IK^T Wt'_{I-1} for the next panel's Wt'
// (the next trailing matrix is A2 without its first block row and column).
// The updated block is in the MFMA output layout, which serves directly as
// the A operand of the next product with inner index k_s(l) = orow(l, s).
template <int PREC>
__device__ __forceinline__ void fused_pass(BatchLds &L, const Lane &q, double *A2, int lda,
                                           int j, const double *Vc, const double *Wc,
                                           const double *Wtn) {
  const int nbk = (j + kBN - 1) / kBN;
  const int ncol = nbk - 1;
  const v4d z64 = {0.0, 0.0, 0.0, 0.0};
  const v4f z32 = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int t = q.tid; t < ncol * kBN * kBN; t += kBT) L.X[t] = 0.0;
  __syncthreads();
  double *tile = L.scr[q.wave];
  for (int kk = q.wave; kk < ncol + kBW; kk += kBW) {
    const int K1 = snake(kk);
    if (K1 >= ncol) continue;
    const int K = K1 + 1;
    double vk[4], wk[4], wtk[4];
    load_vw(Vc, Wc, K, q.l16, q.l4, vk, wk);
#pragma unroll
    for (int s = 0; s < 4; ++s) wtk[s] = gld(Wtn, (K1 * kBN + orow<PREC>(q.lane, s)) * kBN + q.l16);
    v4d xk = z64;
    v4f xk32 = z32;
    auto body = [&](int I, const UpdStage &S) {
      double an[4];
      upd_block<PREC>(q, A2, lda, j, I, K, vk, wk, S, an);
      // block through the per-wave tile: tile[c*17 + r] = A_IK(r, c)
#pragma unroll
      for (int e = 0; e < 4; ++e) tile[orow<PREC>(q.lane, e) * kTS + q.l16] = an[e];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double at[4];  // A_IK(k_s, l%16)
#pragma unroll
      for (int s = 0; s < 4; ++s) at[s] = tile[q.l16 * kTS + orow<PREC>(q.lane, s)];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (I == K) {
        // diagonal block: the upper triangle is the mirror of the lower one
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int rr = q.l16, cc = orow<PREC>(q.lane, e);
          if (rr < cc) an[e] = at[e];
        }
      }
      v4d x = z64;
      v4f x32 = z32;
      mma16<PREC>(x, x32, an, wtk);
      if (I > K) mma16<PREC>(xk, xk32, at, S.t);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        atomicAdd(&L.X[((I - 1) * kBN + orow<PREC>(q.lane, e)) * kBN + q.l16], accv<PREC>(x, x32, e));
    };
    // three blocks in flight
    UpdStage S0, S1, S2;
    load_upd<PREC, true>(q, A2, lda, j, Vc, Wc, Wtn, K, K, S0);
    load_upd<PREC, true>(q, A2, lda, j, Vc, Wc, Wtn, min(K + 1, nbk - 1), K, S1);
    for (int I = K; I < nbk; I += 3) {
      load_upd<PREC, true>(q, A2, lda, j, Vc, Wc, Wtn, min(I + 2, nbk - 1), K, S2);
      body(I, S0);
      if (I + 1 >= nbk) break;
      load_upd<PREC, true>(q, A2, lda, j, Vc, Wc, Wtn, min(I + 3, nbk - 1), K, S0);
      body(I + 1, S1);
      if (I + 2 >= nbk) break;
      load_upd<PREC, true>(q, A2, lda, j, Vc, Wc, Wtn, min(I + 4, nbk - 1), K, S1);
      body(I + 2, S2);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      atomicAdd(&L.X[(K1 * kBN + orow<PREC>(q.lane, e)) * kBN + q.l16], accv<PREC>(xk, xk32, e));
  }
  __syncthreads();
}

template <int PREC>
__global__ __launch_bounds__(kBT) void k_batched(BatchDesc d) {
  __shared__ BatchLds L;
  Lane q;
  q.tid = threadIdx.x;
  q.lane = q.tid & 63;
  q.wave = q.tid >> 6;
  q.l16 = q.lane & 15;
  q.l4 = q.lane >> 4;
  double *Vbuf[2];
  Vbuf[0] = d.ws + (int64_t)blockIdx.x * d.ws_stride;
  Vbuf[1] = Vbuf[0] + kPanelD;
  double *Wc = Vbuf[1] + kPanelD;
  double *Wt = Wc + kPanelD;
  const int w = d.w, b = d.b;
  const bool fuse = (w == kBN && b == kBN);

  for (;;) {
    __syncthreads();
    if (q.tid == 0) L.item = (int)atomicAdd(d.queue, 1u);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(L.item);  // uniform: table entry in SGPRs
    if (it >= d.count) break;
    const BatchEntry ent = d.table[it];
    const int n = ent.n;
    if (n <= w) continue;
    double *A = ent.A;
    const int lda = (int)ent.lda;  // lda * n < 2^29 (host check)
    for (int t = q.tid; t < n - w; t += kBT) gst(ent.tau, t, 0.0);
    const int nref = n - w - 1;
    if (nref <= 0) continue;
    // Each step factors panel c, forms its X (alone, or fused with the
    // previous panel's update of the trailing blocks), forms W and applies
    // the update (all of it, or only the first column block when the next
    // step fuses the rest).  One call site per phase keeps the code small.
    int cur = 0, jp = 0;
    double *A2p = nullptr;
    for (int c = 0;; ) {
      // an opaque copy of lda per panel: keeps the compiler from hoisting
      // lda-derived per-lane offsets out of the panel loop (they would stay
      // live, and spill, across the whole matrix)
      int ldp = __builtin_amdgcn_readfirstlane(lda);
      asm volatile("" : "+s"(ldp));
      const int pb = min(b, nref - c);
      const int r = c + w, j = n - r;
      double *A2 = A + r + (int64_t)r * ldp;
      double *Vc = Vbuf[cur];
      factor_panel(L, q, A + r + (int64_t)c * ldp, ldp, j, pb, ent.tau + c, Vc, Wt);
      if (w > pb) update_a1(L, q, A + r + (int64_t)(c + pb) * ldp, ldp, j, w - pb, Vc, Wt);
      if (A2p && fuse)
        fused_pass<PREC>(L, q, A2p, ldp, jp, Vbuf[cur ^ 1], Wc, Wt);
      else
        x_pass<PREC>(L, q, A2, ldp, j, Wt);
      form_w(L, q, j, Vc, Wt, Wc);
      const int cn = c + pb;
      if (cn >= nref || !fuse)
        syr2k_pass<PREC>(q, A2, ldp, j, Vc, Wc);
      else
        syr2k_col0<PREC>(q, A2, ldp, j, Vc, Wc);
      if (cn >= nref) break;
      A2p = A2;
      jp = j;
      cur ^= 1;
      c = cn;
    }
  }
}

int64_t batched_ws_doubles() { return 4 * kPanelD; }
int batched_max_trailing() { return kBJMax; }
int batched_max_block() { return kBN; }

int launch_batched(int prec, const BatchEntry *table, int count, int w, int b, unsigned *queue,
                   double *ws, int nwg, hipStream_t s) {
  if (count <= 0 || nwg <= 0) return 0;
  if (b < 1 || b > kBN || w < b) return BANDRED_ERR_UNSUPPORTED;
  BatchDesc d{};
  d.table = table;
  d.count = count;
  d.w = w;
  d.b = b;
  d.queue = queue;
  d.ws = ws;
  d.ws_stride = batched_ws_doubles();
  if (prec == P_F64)
    hipLaunchKernelGGL(k_batched<P_F64>, dim3(nwg), dim3(kBT), 0, s, d);
  else
    hipLaunchKernelGGL(k_batched<P_F32>, dim3(nwg), dim3(kBT), 0, s, d);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace br
