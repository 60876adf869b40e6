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
// Products run on 16 x 16 x 4 MFMA blocks: FP64, or FP32 for the trailing
// products 4 and 6 in the FP32-update form.  V and W live in a per-workgroup
// scratch column-major and Wt row-major, rows padded to a multiple of 16, so
// that every operand fragment of the O(j^2) steps 4 and 6 is read with 16
// consecutive lanes on 16 consecutive doubles.  In 4 and 6 each wave owns
// whole column blocks (dealt in snake order) and loads the next block's
// operands before it uses the current ones.
#include "common.hpp"

namespace br {

constexpr int kBT = 512;              // threads per workgroup (8 waves)
constexpr int kBW = kBT / 64;         // waves
constexpr int kBN = 16;               // panel width of the batched path
constexpr int kRPT = 2;               // panel rows per thread
constexpr int kBJMax = kBT * kRPT;    // largest trailing order j = n - w

struct BatchDesc {
  const BatchEntry *table;
  int count;
  int w, b;
  unsigned *queue;
  double *ws;          // per-workgroup scratch: V, W, Wt, each kBJMax x 16
  int64_t ws_stride;   // doubles per workgroup
};

template <int PREC>
__device__ __forceinline__ int orow(int lane, int e) {
  return (PREC == P_F64) ? (lane >> 4) + 4 * e : 4 * (lane >> 4) + e;
}

// acc += A B for 16 x 16 blocks with inner dimension 16;
// a[s] = A(l%16, l/16 + 4s), b[s] = B(l/16 + 4s, l%16)  (l = lane)
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

// Sum of 16 per-lane values over the wave by recursive halving: at each step a
// lane keeps half of its values and receives the partner's copy of that half.
// On return lane l holds the total of value sum16_index(l).
__device__ __forceinline__ double wave_sum16(const double (&v)[kBN], int lane) {
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
  double h8[8], h4[4], h2[2];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const double keep = b5 ? v[8 + t] : v[t], send = b5 ? v[t] : v[8 + t];
    h8[t] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const double keep = b4 ? h8[4 + t] : h8[t], send = b4 ? h8[t] : h8[4 + t];
    h4[t] = keep + __shfl_xor(send, 16, 64);
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const double keep = b3 ? h4[2 + t] : h4[t], send = b3 ? h4[t] : h4[2 + t];
    h2[t] = keep + __shfl_xor(send, 8, 64);
  }
  double h1 = (b2 ? h2[1] : h2[0]) + __shfl_xor(b2 ? h2[0] : h2[1], 4, 64);
  h1 += __shfl_xor(h1, 2, 64);
  h1 += __shfl_xor(h1, 1, 64);
  return h1;
}

__device__ __forceinline__ int sum16_index(int lane) {
  return ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
}

struct BatchLds {
  double X[kBJMax * kBN];        // X accumulator, row-major j x 16
  double scr[kBW][kBN * kBN];    // per-wave partial products / transpose tiles
  double S[kBN * kBN], T[kBN * kBN], M[kBN * kBN];
  double red[kBW][kBN];          // per-wave column sums
  double tot[kBN];               // column sums of the workgroup
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
// panel a[][] is never indexed dynamically): one workgroup reduction gives the
// sums s_k = sum_{rho > I} a(rho, I) a(rho, k) and the pivot row; every thread
// then forms the reflector and updates its rows of the trailing columns.
template <int I>
__device__ __forceinline__ void house_col(double (&a)[kRPT][kBN], BatchLds &L, int tid, int lane,
                                          int wave, int pb, double *tau_out) {
  if (I >= pb) return;
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
  if ((lane & 3) == 0) L.red[wave][sum16_index(lane)] = q;
  if (tid == I) {
#pragma unroll
    for (int k = 0; k < kBN; ++k) L.prow[I & 1][k] = a[0][k];
  }
  __syncthreads();
  if (tid < kBN) {
    double s = 0.0;
#pragma unroll
    for (int q2 = 0; q2 < kBW; ++q2) s += L.red[q2][tid];
    L.tot[tid] = s;
  }
  __syncthreads();
  // reflector: beta = -sign(alpha) ||(alpha, x)||, v = x / (alpha - beta)
  const double alpha = L.prow[I & 1][I], sig2 = L.tot[I];
  double tau = 0.0, dv = 0.0, beta = alpha;
  if (sig2 != 0.0) {
    const double nrm = sqrt(alpha * alpha + sig2);
    beta = (alpha < 0.0) ? nrm : -nrm;
    tau = (beta - alpha) / beta;
    dv = 1.0 / (alpha - beta);
  }
  if (tau != 0.0) {
    // column k: a_k -= tau v (v^T a_k) with v^T a_k = p_k + s_k / (alpha - beta)
    double f[kBN];
#pragma unroll
    for (int k = I + 1; k < kBN; ++k) f[k] = tau * (L.prow[I & 1][k] + L.tot[k] * dv);
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
    tau_out[I] = tau;
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

template <int PREC>
__global__ __launch_bounds__(kBT) void k_batched(BatchDesc d) {
  __shared__ BatchLds L;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  // scratch: V and W column-major (ld kBJMax), Wt = V T row-major (16 columns)
  double *Vc = d.ws + (int64_t)blockIdx.x * d.ws_stride;
  double *Wc = Vc + (int64_t)kBJMax * kBN;
  double *Wt = Wc + (int64_t)kBJMax * kBN;
  const int w = d.w, b = d.b;
  const v4d z64 = {0.0, 0.0, 0.0, 0.0};
  const v4f z32 = {0.0f, 0.0f, 0.0f, 0.0f};

  for (;;) {
    __syncthreads();
    if (tid == 0) L.item = (int)atomicAdd(d.queue, 1u);
    __syncthreads();
    const int it = L.item;
    if (it >= d.count) break;
    const BatchEntry ent = d.table[it];
    const int n = ent.n;
    if (n <= w) continue;
    double *A = ent.A;
    const int64_t lda = ent.lda;
    for (int q = tid; q < n - w; q += kBT) ent.tau[q] = 0.0;
    const int nref = n - w - 1;
    for (int c = 0; c < nref; c += b) {
      const int pb = min(b, nref - c);
      const int r = c + w, j = n - r;
      const int nbk = (j + kBN - 1) / kBN;
      double *P = A + r + (int64_t)c * lda;

      // ---- 1. panel QR, rows tid + kBT*s of the panel in registers ----
      double a[kRPT][kBN];
#pragma unroll
      for (int s = 0; s < kRPT; ++s) {
        const int rho = tid + kBT * s;
#pragma unroll
        for (int k = 0; k < kBN; ++k) a[s][k] = (rho < j && k < pb) ? P[rho + (int64_t)k * lda] : 0.0;
      }
      ColLoop<0>::run(a, L, tid, lane, wave, pb, ent.tau + c);
      // panel back in place; explicit V (unit diagonal, zeros above and in
      // the padding rows and columns)
#pragma unroll
      for (int s = 0; s < kRPT; ++s) {
        const int rho = tid + kBT * s;
        if (rho < j) {
#pragma unroll
          for (int k = 0; k < kBN; ++k)
            if (k < pb) P[rho + (int64_t)k * lda] = a[s][k];
        }
        if (rho < nbk * kBN) {
#pragma unroll
          for (int k = 0; k < kBN; ++k) {
            double v = 0.0;
            if (k < pb && rho < j) v = (rho == k) ? 1.0 : (rho > k ? a[s][k] : 0.0);
            Vc[(int64_t)k * kBJMax + rho] = v;
          }
        }
      }
      __syncthreads();

      // ---- 2. S = V^T V; T; Wt = V T ----
      {
        v4d acc = z64;
        v4f acc32 = z32;
        for (int I = wave; I < nbk; I += kBW) {
          double av[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) av[s] = Vc[(int64_t)l16 * kBJMax + I * kBN + l4 + 4 * s];
          mma16<P_F64>(acc, acc32, av, av);  // V^T(l%16, k) and V(k, l%16) are the same value
        }
        reduce_waves(L, acc, L.S, tid, lane, wave);
      }
      if (wave == 0) {
        // T(i,i) = tau_i, T(0:i, i) = -tau_i T(0:i, 0:i) S(0:i, i); lane l
        // holds row l of T
        double trow[kBN];
#pragma unroll
        for (int i = 0; i < kBN; ++i) {
          double acc = 0.0;
#pragma unroll
          for (int m = 0; m < i; ++m) acc += trow[m] * L.S[m * kBN + i];
          const double ti = (i < pb) ? L.tau[i] : 0.0;
          trow[i] = (lane < i) ? -ti * acc : (lane == i ? ti : 0.0);
        }
        if (lane < kBN) {
#pragma unroll
          for (int i = 0; i < kBN; ++i) L.T[lane * kBN + i] = trow[i];
        }
      }
      __syncthreads();
      for (int I = wave; I < nbk; I += kBW) {
        v4d acc = z64;
        v4f acc32 = z32;
        double av[4], bv[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          av[s] = Vc[(int64_t)(l4 + 4 * s) * kBJMax + I * kBN + l16];
          bv[s] = L.T[(l4 + 4 * s) * kBN + l16];
        }
        mma16<P_F64>(acc, acc32, av, bv);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          Wt[(int64_t)(I * kBN + orow<P_F64>(lane, e)) * kBN + l16] = acc[e];
      }
      __syncthreads();

      // ---- 3. A1 -= V (Wt^T A1), 16 columns at a time ----
      const int a1w = w - pb;
      if (a1w > 0) {
        double *A1 = A + r + (int64_t)(c + pb) * lda;
        const int nq = (a1w + kBN - 1) / kBN;
        for (int Q = 0; Q < nq; ++Q) {
          v4d acc = z64;
          v4f acc32 = z32;
          for (int I = wave; I < nbk; I += kBW) {
            double av[4], bv[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              const int row = I * kBN + l4 + 4 * s, col = Q * kBN + l16;
              av[s] = Wt[(int64_t)row * kBN + l16];
              bv[s] = (row < j && col < a1w) ? A1[row + (int64_t)col * lda] : 0.0;
            }
            mma16<P_F64>(acc, acc32, av, bv);
          }
          reduce_waves(L, acc, L.M, tid, lane, wave);  // Z_Q, kept in the M buffer
          for (int I = wave; I < nbk; I += kBW) {
            // D(a, c) = sum_k Z(k, a) V_I(c, k) = (V_I Z)(c, a): lanes run down rows of A1
            v4d o = z64;
            v4f o32 = z32;
            double av[4], bv[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              av[s] = L.M[(l4 + 4 * s) * kBN + l16];
              bv[s] = Vc[(int64_t)(l4 + 4 * s) * kBJMax + I * kBN + l16];
            }
            mma16<P_F64>(o, o32, av, bv);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int row = I * kBN + l16, col = Q * kBN + orow<P_F64>(lane, e);
              if (row < j && col < a1w) A1[row + (int64_t)col * lda] -= o[e];
            }
          }
          __syncthreads();
        }
      }

      // ---- 4. X = A2 Wt from the lower blocks of A2 ----
      // Wave-owned column blocks K in snake order (column K holds nbk - K
      // blocks); the next block's operands are loaded before the current
      // block is used.
      double *A2 = A + r + (int64_t)r * lda;
      for (int q = tid; q < nbk * kBN * kBN; q += kBT) L.X[q] = 0.0;
      __syncthreads();
      {
        double *tile = L.scr[wave];
        for (int kk = wave; kk < nbk + kBW; kk += kBW) {
          const int round = kk / kBW, pos = kk % kBW;
          const int K = round * kBW + ((round & 1) ? kBW - 1 - pos : pos);
          if (K >= nbk) continue;
          v4d xk = z64;
          v4f xk32 = z32;
          double wtk[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) wtk[s] = Wt[(int64_t)(K * kBN + l4 + 4 * s) * kBN + l16];
          // lane l holds A_IK(l%16, l/16 + 4s); the diagonal block is mirrored
          auto load_blk = [&](int I, double (&ak)[4], double (&wti)[4]) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              const int row = I * kBN + l16, col = K * kBN + l4 + 4 * s;
              double v = 0.0;
              if (row < j && col < j)
                v = (row >= col) ? A2[row + (int64_t)col * lda] : A2[col + (int64_t)row * lda];
              ak[s] = v;
              wti[s] = Wt[(int64_t)(I * kBN + l4 + 4 * s) * kBN + l16];
            }
          };
          double ak[4], wti[4];
          load_blk(K, ak, wti);
          for (int I = K; I < nbk; ++I) {
            double akn[4], wtin[4];
            if (I + 1 < nbk) load_blk(I + 1, akn, wtin);
            v4d o = z64;
            v4f o32 = z32;
            mma16<PREC>(o, o32, ak, wtk);
#pragma unroll
            for (int e = 0; e < 4; ++e)
              atomicAdd(&L.X[(I * kBN + orow<PREC>(lane, e)) * kBN + l16], accv<PREC>(o, o32, e));
            if (I > K) {
#pragma unroll
              for (int s = 0; s < 4; ++s) tile[(l4 + 4 * s) * kBN + l16] = ak[s];
              __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
              __builtin_amdgcn_wave_barrier();
              __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
              double at[4];
#pragma unroll
              for (int s = 0; s < 4; ++s) at[s] = tile[l16 * kBN + l4 + 4 * s];  // A_IK(l/16 + 4s, l%16)
              __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
              __builtin_amdgcn_wave_barrier();
              __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
              mma16<PREC>(xk, xk32, at, wti);
            }
            if (I + 1 < nbk) {
#pragma unroll
              for (int s = 0; s < 4; ++s) {
                ak[s] = akn[s];
                wti[s] = wtin[s];
              }
            }
          }
#pragma unroll
          for (int e = 0; e < 4; ++e)
            atomicAdd(&L.X[(K * kBN + orow<PREC>(lane, e)) * kBN + l16], accv<PREC>(xk, xk32, e));
        }
      }
      __syncthreads();

      // ---- 5. M = Wt^T X; W = X - 1/2 V M (stored column-major) ----
      {
        v4d acc = z64;
        v4f acc32 = z32;
        for (int I = wave; I < nbk; I += kBW) {
          double av[4], bv[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int row = I * kBN + l4 + 4 * s;
            av[s] = Wt[(int64_t)row * kBN + l16];
            bv[s] = L.X[row * kBN + l16];
          }
          mma16<P_F64>(acc, acc32, av, bv);
        }
        reduce_waves(L, acc, L.M, tid, lane, wave);
      }
      for (int I = wave; I < nbk; I += kBW) {
        v4d o = z64;
        v4f o32 = z32;
        double av[4], bv[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          av[s] = Vc[(int64_t)(l4 + 4 * s) * kBJMax + I * kBN + l16];
          bv[s] = L.M[(l4 + 4 * s) * kBN + l16];
        }
        mma16<P_F64>(o, o32, av, bv);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = I * kBN + orow<P_F64>(lane, e);
          Wc[(int64_t)l16 * kBJMax + row] = L.X[row * kBN + l16] - 0.5 * o[e];
        }
      }
      __syncthreads();

      // ---- 6. A2 -= W V^T + V W^T on the lower blocks ----
      // Wave-owned column blocks as in 4: V_K, W_K stay in registers,
      // the next row block's operands are loaded ahead.
      for (int kk = wave; kk < nbk + kBW; kk += kBW) {
        const int round = kk / kBW, pos = kk % kBW;
        const int K = round * kBW + ((round & 1) ? kBW - 1 - pos : pos);
        if (K >= nbk) continue;
        // A operands: V_K(a, k), W_K(a, k) with a = l%16, k = l/16 + 4s
        double vk[4], wk[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          vk[s] = Vc[(int64_t)(l4 + 4 * s) * kBJMax + K * kBN + l16];
          wk[s] = Wc[(int64_t)(l4 + 4 * s) * kBJMax + K * kBN + l16];
        }
        // B operands W_I(c, k), V_I(c, k) with c = l%16; lane holds
        // A2(I*16 + c, K*16 + orow(e))
        auto load_blk = [&](int I, double (&wi)[4], double (&vi)[4], double (&ai)[4]) {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            wi[s] = Wc[(int64_t)(l4 + 4 * s) * kBJMax + I * kBN + l16];
            vi[s] = Vc[(int64_t)(l4 + 4 * s) * kBJMax + I * kBN + l16];
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int row = I * kBN + l16, col = K * kBN + orow<PREC>(lane, e);
            ai[e] = (row < j && row >= col) ? A2[row + (int64_t)col * lda] : 0.0;
          }
        };
        double wi[4], vi[4], ai[4];
        load_blk(K, wi, vi, ai);
        for (int I = K; I < nbk; ++I) {
          double win[4], vin[4], ain[4];
          if (I + 1 < nbk) load_blk(I + 1, win, vin, ain);
          // D(a, c) = sum_k V_K(a, k) W_I(c, k) + W_K(a, k) V_I(c, k)
          v4d o = z64;
          v4f o32 = z32;
          mma16<PREC>(o, o32, vk, wi);
          mma16<PREC>(o, o32, wk, vi);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int row = I * kBN + l16, col = K * kBN + orow<PREC>(lane, e);
            if (row < j && row >= col) A2[row + (int64_t)col * lda] = ai[e] - accv<PREC>(o, o32, e);
          }
          if (I + 1 < nbk) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              wi[s] = win[s];
              vi[s] = vin[s];
              ai[s] = ain[s];
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

int64_t batched_ws_doubles() { return (int64_t)3 * kBJMax * kBN; }
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
