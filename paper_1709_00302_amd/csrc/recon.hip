// recon.hip -- panel factorisation by CholeskyQR2 plus Householder
// reconstruction (gfx950).
//
// The panel P (m x b, b <= 128) is factored as P = Q R by two CholeskyQR
// passes (G = P^T P = R1^T R1, Q1 = P R1^-1, Q1^T Q1 = R2^T R2,
// Q = Q1 R2^-1, R = R2 R1); the Householder vectors of the same panel are
// then rebuilt from Q as in Ballard et al. (the reconstruction the paper cites
// as the way around tile kernels, Sec. 2.2): with the sign matrix S chosen on
// the fly as S_k = -sign of the current pivot, the LU factorisation without
// pivoting Q(0:b, :) - S = L U gives
//     V = [L; Q(b:m, :) U^-1],   T = -U S L^-T,   R_householder = S R,
// which in exact arithmetic is exactly what column-by-column Householder QR
// with beta = -sign(alpha) ||x|| produces (LAPACK's sign convention), so the
// stored reflectors and tau are those of the unblocked reduction.  The
// bottom rows are formed as V(b:m, :) = Q1(b:m, :) (R2^-1 U^-1).
//
// The O(m b^2) products run on the MFMA GEMM kernel; the O(b^3) sequential
// factorisations run here in one workgroup of 1024 threads.  Each thread keeps
// a 4 x 4 tile of the b x b matrix in registers (32 x 32 tiles cover
// b = 128; sizes below 128 are padded with the identity, which every
// operation below leaves invariant).  The factorisations are blocked by 4 and
// take one workgroup barrier per block step: the diagonal block and its block
// row are handled by the wave that owns them (broadcasts from the diagonal
// tile's lane through the scalar unit), the block row and column are
// published through LDS, and every trailing tile takes one rank-4 update.
// What other threads need of a diagonal block is either fixed in advance
// (diagonal blocks of a triangular matrix, stored once) or recomputed by each
// thread from the published raw block.
//
// Rank-deficient or structurally reduced panels: a pivot of the first
// Cholesky below rel * (original diagonal), or a panel with no nonzero below
// its diagonal, raises a device flag; the remaining kernels of this path then
// return at once and the exact per-column Householder kernel takes the panel.
#include "common.hpp"

namespace br {

constexpr int kRT = 1024;          // threads of the register-tiled kernels
constexpr int kTE = 4;             // tile edge
constexpr int kNTl = kNbMax / kTE;  // tiles per edge (32)

struct Tile {
  double a[kTE][kTE];
};

// thread t owns tile (bi, bj) = (t / 32, t % 32); tile row i lives in wave
// i / 2, tile (i, j) in lane 32 (i % 2) + j of that wave
struct TileCtx {
  int t, bi, bj, lane;
};

__device__ __forceinline__ TileCtx tile_ctx() {
  TileCtx c;
  c.t = threadIdx.x;
  c.bi = c.t >> 5;
  c.bj = c.t & 31;
  c.lane = c.t & 63;
  return c;
}

__device__ __forceinline__ int diag_lane(int kb) { return 32 * (kb & 1) + kb; }

// Value of x in lane l of the wave (l uniform), through the scalar unit.
__device__ __forceinline__ double bcast_lane(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// 1/x and 1/sqrt(x) from the hardware approximations plus two Newton steps
// (each step squares the relative error): accurate to a few units in the last
// place, and far shorter dependence chains than the correctly rounded
// division and square root, which sit on the sequential pivot chain here.
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

// Shared buffers of the blocked steps (double buffered by block parity).
// The block row / column buffers double as the staging area of coalesced
// tile loads and stores (32 columns of 128 rows at a time).
struct Bcast {
  union {
    struct {
      double rb[2][kTE][kNbMax];  // a block row (4 rows)
      double cb[2][kNbMax][kTE];  // a block column (4 columns)
    };
    double stage[32 * kNbMax];
  };
  double dg[kNTl][kTE * kTE];   // per-block data fixed during a sweep
  double pb[2][kTE * kTE];      // the current diagonal block
  double d0[kNbMax];            // original diagonal (Cholesky breakdown test)
  double sg[kNbMax];            // LU signs
  int bad;
};

// load a b x b column-major matrix (identity-padded to 128 x 128): every
// global load is issued before the first wait (one memory latency), then the
// tiles are redistributed through LDS 32 columns at a time
__device__ __forceinline__ void tile_load(Tile &T, const TileCtx &c, Bcast &s, const double *G,
                                          int ld, int b) {
  constexpr int E = 32 * kNbMax / kRT;  // elements per thread per chunk
  double v[4][E];
#pragma unroll
  for (int ch = 0; ch < 4; ++ch)
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int e = c.t + kRT * k;
      const int i = e & (kNbMax - 1), j = 32 * ch + (e >> 7);
      v[ch][k] = (i < b && j < b) ? G[i + (int64_t)j * ld] : (i == j ? 1.0 : 0.0);
    }
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) s.stage[c.t + kRT * k] = v[ch][k];
    __syncthreads();
    if ((c.bj >> 3) == ch) {
      const int j0 = kTE * (c.bj & 7);
#pragma unroll
      for (int r = 0; r < kTE; ++r)
#pragma unroll
        for (int q = 0; q < kTE; ++q) T.a[r][q] = s.stage[(j0 + q) * kNbMax + kTE * c.bi + r];
    }
  }
  __syncthreads();
}

// store (parts of) the tile straight from the registers: mode 0 all, 1 upper
// (zeros below), 2 unit lower (ones on the diagonal, zeros above)
__device__ __forceinline__ void tile_store(const Tile &T, const TileCtx &c, Bcast &, double *G,
                                           int64_t ld, int b, int mode) {
#pragma unroll
  for (int q = 0; q < kTE; ++q)
#pragma unroll
    for (int r = 0; r < kTE; ++r) {
      const int i = kTE * c.bi + r, j = kTE * c.bj + q;
      double v = T.a[r][q];
      if (mode == 1 && j < i) v = 0.0;
      if (mode == 2) v = (i == j) ? 1.0 : (i > j ? v : 0.0);
      if (i < b && j < b) G[i + (int64_t)j * ld] = v;
    }
}

// Blocked upper Cholesky in place: G = R^T R, R in the upper triangle.  The
// block row kb is factored by its owners (one wave) with the diagonal tile's
// values broadcast from its lane; the trailing upper tiles then take one
// rank-4 update.  Returns false (in every thread) on a pivot <= rel * d0[k].
__device__ __forceinline__ bool blk_chol(Tile &T, const TileCtx &c, Bcast &s, int b, double rel) {
  if (c.t == 0) s.bad = 0;
  __syncthreads();
  const int nblk = (b + kTE - 1) / kTE;
  for (int kb = 0; kb < nblk; ++kb) {
    const int buf = kb & 1;
    if (c.bi == kb && c.bj >= kb) {
      const int dl = diag_lane(kb);
      const bool diag = (c.bj == kb);
      bool ok = true;
#pragma unroll
      for (int kr = 0; kr < kTE; ++kr) {
        const double d = bcast_lane(T.a[kr][kr], dl);
        ok = ok && (d > rel * s.d0[kTE * kb + kr]);
        const double ir = rsq_nr(d > 0.0 ? d : 1.0), r = (d > 0.0 ? d : 1.0) * ir;
#pragma unroll
        for (int q = 0; q < kTE; ++q) {
          if (!diag || q > kr) T.a[kr][q] *= ir;
          else if (q == kr) T.a[kr][q] = r;
        }
#pragma unroll
        for (int k2 = kr + 1; k2 < kTE; ++k2) {
          const double f = bcast_lane(T.a[kr][k2], dl);
#pragma unroll
          for (int q = 0; q < kTE; ++q) T.a[k2][q] -= f * T.a[kr][q];
        }
      }
#pragma unroll
      for (int kr = 0; kr < kTE; ++kr)
#pragma unroll
        for (int q = 0; q < kTE; ++q) s.rb[buf][kr][kTE * c.bj + q] = T.a[kr][q];
      if (diag && !ok) s.bad = 1;
    }
    __syncthreads();
    if (s.bad) return false;
    if (c.bi > kb && c.bj >= c.bi) {
#pragma unroll
      for (int l = 0; l < kTE; ++l) {
        double x[kTE], y[kTE];
#pragma unroll
        for (int r = 0; r < kTE; ++r) x[r] = s.rb[buf][l][kTE * c.bi + r];
#pragma unroll
        for (int q = 0; q < kTE; ++q) y[q] = s.rb[buf][l][kTE * c.bj + q];
#pragma unroll
        for (int r = 0; r < kTE; ++r)
#pragma unroll
          for (int q = 0; q < kTE; ++q) T.a[r][q] -= x[r] * y[q];
      }
    }
  }
  __syncthreads();
  return true;
}

// In-place inverse of the 4 x 4 upper triangular block a (zeros below).
__device__ __forceinline__ void inv4_upper(double (&a)[kTE][kTE]) {
#pragma unroll
  for (int i = kTE - 1; i >= 0; --i) {
    const double ii = 1.0 / a[i][i];
#pragma unroll
    for (int j = kTE - 1; j > i; --j) {
      double acc = 0.0;
#pragma unroll
      for (int l = i + 1; l <= j; ++l) acc += a[i][l] * a[l][j];
      a[i][j] = -acc * ii;
    }
    a[i][i] = ii;
#pragma unroll
    for (int j = 0; j < i; ++j) a[i][j] = 0.0;
  }
}

// Blocked in-place Gauss-Jordan inverse of an upper triangular matrix.
// Pivot block kb: A_kk <- A_kk^-1, A_kj <- A_kk^-1 A_kj, A_ik <- -A_ik A_kk^-1
// and A_ij -= A_ik(old) A_kj(new) for i < k < j.  A diagonal block is never
// touched before its own step, so all the A_kk^-1 are formed up front (by the
// diagonal owners, into LDS) and each step needs a single barrier.
__device__ __forceinline__ void blk_inv_upper(Tile &T, const TileCtx &c, Bcast &s, int b) {
  const int nblk = (b + kTE - 1) / kTE;
  if (c.bi == c.bj) {
    inv4_upper(T.a);
#pragma unroll
    for (int r = 0; r < kTE; ++r)
#pragma unroll
      for (int q = 0; q < kTE; ++q) s.dg[c.bi][kTE * r + q] = T.a[r][q];
  }
  __syncthreads();
  for (int kb = 0; kb < nblk; ++kb) {
    const int buf = kb & 1;
    double P[kTE * kTE];
    if ((c.bi == kb && c.bj > kb) || (c.bj == kb && c.bi < kb)) {
#pragma unroll
      for (int e = 0; e < kTE * kTE; ++e) P[e] = s.dg[kb][e];
    }
    if (c.bi == kb && c.bj > kb) {  // A_kj <- P A_kj, rows top-down in place
#pragma unroll
      for (int r = 0; r < kTE; ++r)
#pragma unroll
        for (int q = 0; q < kTE; ++q) {
          double acc = 0.0;
#pragma unroll
          for (int l = r; l < kTE; ++l) acc += P[kTE * r + l] * T.a[l][q];
          T.a[r][q] = acc;
        }
#pragma unroll
      for (int r = 0; r < kTE; ++r)
#pragma unroll
        for (int q = 0; q < kTE; ++q) s.rb[buf][r][kTE * c.bj + q] = T.a[r][q];
    }
    if (c.bj == kb && c.bi < kb) {  // publish A_ik(old); A_ik <- -A_ik P
#pragma unroll
      for (int r = 0; r < kTE; ++r)
#pragma unroll
        for (int q = 0; q < kTE; ++q) s.cb[buf][kTE * c.bi + r][q] = T.a[r][q];
#pragma unroll
      for (int q = kTE - 1; q >= 0; --q)
#pragma unroll
        for (int r = 0; r < kTE; ++r) {
          double acc = 0.0;
#pragma unroll
          for (int l = 0; l <= q; ++l) acc += T.a[r][l] * P[kTE * l + q];
          T.a[r][q] = -acc;
        }
    }
    __syncthreads();
    if (c.bi < kb && c.bj > kb) {
#pragma unroll
      for (int l = 0; l < kTE; ++l) {
        double x[kTE], y[kTE];
#pragma unroll
        for (int r = 0; r < kTE; ++r) x[r] = s.cb[buf][kTE * c.bi + r][l];
#pragma unroll
        for (int q = 0; q < kTE; ++q) y[q] = s.rb[buf][l][kTE * c.bj + q];
#pragma unroll
        for (int r = 0; r < kTE; ++r)
#pragma unroll
          for (int q = 0; q < kTE; ++q) T.a[r][q] -= x[r] * y[q];
      }
    }
  }
  __syncthreads();
}

// Blocked LU without pivoting of (W - S), S_k = -sign of the current pivot
// (chosen on the fly).  L (unit, strict lower) and U (upper) overwrite the
// tiles; the signs go to s.sg.  Step kb: the block row (diagonal LU and
// U_kj = L_kk^-1 A_kj) in its wave; the block column publishes its raw
// tiles; after the barrier every thread of a lower block row forms
// L_ik = A_ik U_kk^-1 itself and applies the rank-4 update.
__device__ __forceinline__ void blk_lu_sign(Tile &T, const TileCtx &c, Bcast &s, int b) {
  const int nblk = (b + kTE - 1) / kTE;
  for (int kb = 0; kb < nblk; ++kb) {
    const int buf = kb & 1;
    if (c.bi == kb && c.bj >= kb) {
      const int dl = diag_lane(kb);
      const bool diag = (c.bj == kb);
#pragma unroll
      for (int kr = 0; kr < kTE; ++kr) {
        const double w = bcast_lane(T.a[kr][kr], dl);
        const double sgn = (w >= 0.0) ? -1.0 : 1.0;
        const double piv = w - sgn;  // |piv| >= 1
        const double ip = rcp_nr(piv);
        if (diag) {
          T.a[kr][kr] = piv;
#pragma unroll
          for (int i = kr + 1; i < kTE; ++i) T.a[i][kr] *= ip;
          if (c.lane == dl) s.sg[kTE * kb + kr] = sgn;
        }
#pragma unroll
        for (int i = kr + 1; i < kTE; ++i) {
          const double l = bcast_lane(T.a[i][kr], dl);  // L(i, kr) of the diagonal block
#pragma unroll
          for (int q = 0; q < kTE; ++q)
            if (!diag || q > kr) T.a[i][q] -= l * T.a[kr][q];
        }
      }
      if (diag) {
#pragma unroll
        for (int r = 0; r < kTE; ++r)
#pragma unroll
          for (int q = 0; q < kTE; ++q) s.pb[buf][kTE * r + q] = T.a[r][q];
      } else {
#pragma unroll
        for (int r = 0; r < kTE; ++r)
#pragma unroll
          for (int q = 0; q < kTE; ++q) s.rb[buf][r][kTE * c.bj + q] = T.a[r][q];
      }
    }
    if (c.bj == kb && c.bi > kb) {
#pragma unroll
      for (int r = 0; r < kTE; ++r)
#pragma unroll
        for (int q = 0; q < kTE; ++q) s.cb[buf][kTE * c.bi + r][q] = T.a[r][q];
    }
    __syncthreads();
    if (c.bi > kb && c.bj >= kb) {
      // L_ik = A_ik U_kk^-1 from the published raw block
      double U[kTE * kTE], A[kTE][kTE];
#pragma unroll
      for (int e = 0; e < kTE * kTE; ++e) U[e] = s.pb[buf][e];
#pragma unroll
      for (int r = 0; r < kTE; ++r)
#pragma unroll
        for (int q = 0; q < kTE; ++q) A[r][q] = s.cb[buf][kTE * c.bi + r][q];
      double L[kTE][kTE];
#pragma unroll
      for (int q = 0; q < kTE; ++q) {
        const double iu = rcp_nr(U[kTE * q + q]);
#pragma unroll
        for (int r = 0; r < kTE; ++r) {
          double v = A[r][q];
#pragma unroll
          for (int l = 0; l < q; ++l) v -= L[r][l] * U[kTE * l + q];
          L[r][q] = v * iu;
        }
      }
      if (c.bj == kb) {
#pragma unroll
        for (int r = 0; r < kTE; ++r)
#pragma unroll
          for (int q = 0; q < kTE; ++q) T.a[r][q] = L[r][q];
      } else {
#pragma unroll
        for (int l = 0; l < kTE; ++l) {
          double y[kTE];
#pragma unroll
          for (int q = 0; q < kTE; ++q) y[q] = s.rb[buf][l][kTE * c.bj + q];
#pragma unroll
          for (int r = 0; r < kTE; ++r)
#pragma unroll
            for (int q = 0; q < kTE; ++q) T.a[r][q] -= L[r][l] * y[q];
        }
      }
    }
  }
  __syncthreads();
}

// With L (strict lower, unit) and U (upper) in the tiles: T L^T = -U S,
// solved in place over the upper triangle (L is kept), one column block of T
// at a time.  The diagonal blocks of L are stored once; step lb solves the
// column block lb of T against L_ll, publishes it with the L blocks of the
// same block column, and the trailing upper tiles take one rank-4 update.
__device__ __forceinline__ void blk_tsolve(Tile &T, const TileCtx &c, Bcast &s, int b) {
#pragma unroll
  for (int r = 0; r < kTE; ++r)
#pragma unroll
    for (int q = 0; q < kTE; ++q) {
      const int i = kTE * c.bi + r, j = kTE * c.bj + q;
      if (j >= i && j < b) T.a[r][q] = -T.a[r][q] * s.sg[j];
    }
  if (c.bi == c.bj) {
#pragma unroll
    for (int r = 0; r < kTE; ++r)
#pragma unroll
      for (int q = 0; q < kTE; ++q) s.dg[c.bi][kTE * r + q] = T.a[r][q];  // L_ll below the diagonal
  }
  __syncthreads();
  const int nblk = (b + kTE - 1) / kTE;
  for (int lb = 0; lb < nblk; ++lb) {
    const int buf = lb & 1;
    if (c.bj == lb) {
      if (c.bi <= lb) {  // T_il = C_il L_ll^-T (upper part only on the diagonal tile)
        double Ld[kTE * kTE];
#pragma unroll
        for (int e = 0; e < kTE * kTE; ++e) Ld[e] = s.dg[lb][e];
        const bool diag = (c.bi == lb);
#pragma unroll
        for (int q = 0; q < kTE; ++q)
#pragma unroll
          for (int r = 0; r < kTE; ++r) {
            if (diag && r > q) continue;
            double v = T.a[r][q];
#pragma unroll
            for (int l = 0; l < q; ++l)
              if (!diag || l >= r) v -= T.a[r][l] * Ld[kTE * q + l];
            T.a[r][q] = v;
          }
#pragma unroll
        for (int r = 0; r < kTE; ++r)
#pragma unroll
          for (int q = 0; q < kTE; ++q)
            s.cb[buf][kTE * c.bi + r][q] = (diag && r > q) ? 0.0 : T.a[r][q];
      } else {  // L_jl below the diagonal block
#pragma unroll
        for (int r = 0; r < kTE; ++r)
#pragma unroll
          for (int q = 0; q < kTE; ++q) s.cb[buf][kTE * c.bi + r][q] = T.a[r][q];
      }
    }
    __syncthreads();
    if (c.bi <= lb && c.bj > lb) {
      // C_ij -= sum_l T(i, l) L(j, l) over the 4 columns l of block lb
#pragma unroll
      for (int l = 0; l < kTE; ++l) {
        double x[kTE], y[kTE];
#pragma unroll
        for (int r = 0; r < kTE; ++r) x[r] = s.cb[buf][kTE * c.bi + r][l];
#pragma unroll
        for (int q = 0; q < kTE; ++q) y[q] = s.cb[buf][kTE * c.bj + q][l];
#pragma unroll
        for (int r = 0; r < kTE; ++r)
#pragma unroll
          for (int q = 0; q < kTE; ++q) T.a[r][q] -= x[r] * y[q];
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// kernel A: R = chol(G), R^-1 (both full column-major, zeros below)
// flag[0]: raised on breakdown; flag[1]: nonzero count of the panel's
// strictly lower part (0 = structurally reduced panel)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRT) void k_chol_inv(const double *G, int ldg, int b, double rel,
                                                  double *R, double *Rinv, int *flag,
                                                  int check_structure) {
  __shared__ Bcast s;
  if (flag[0]) return;
  if (check_structure && flag[1] == 0) {
    if (threadIdx.x == 0) flag[0] = 1;
    return;
  }
  const TileCtx c = tile_ctx();
  if (c.t < kNbMax) s.d0[c.t] = (c.t < b) ? G[c.t + (int64_t)c.t * ldg] : 1.0;
  Tile T;
  tile_load(T, c, s, G, ldg, b);
  __syncthreads();
  if (!blk_chol(T, c, s, b, rel)) {
    if (c.t == 0) flag[0] = 1;
    return;
  }
  // the upper factor only: zero the strictly lower tiles and parts
#pragma unroll
  for (int r = 0; r < kTE; ++r)
#pragma unroll
    for (int q = 0; q < kTE; ++q)
      if (kTE * c.bj + q < kTE * c.bi + r) T.a[r][q] = 0.0;
  tile_store(T, c, s, R, b, b, 1);
  blk_inv_upper(T, c, s, b);
  tile_store(T, c, s, Rinv, b, b, 1);
}

// ---------------------------------------------------------------------------
// kernel B: Qtop (b x b) -> LU with signs -> V top block (unit lower),
// T = -U S L^-T (and tau), U^-1 (full, zeros below), S
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRT) void k_recon(const double *Qtop, int ldq, int b, double *V,
                                               int64_t ldv, double *Tout, int ldt, double *tau,
                                               double *Uinv, double *sgn, const int *flag) {
  __shared__ Bcast s;
  if (flag[0]) return;
  const TileCtx c = tile_ctx();
  Tile T;
  tile_load(T, c, s, Qtop, ldq, b);
  __syncthreads();
  blk_lu_sign(T, c, s, b);
  tile_store(T, c, s, V, ldv, b, 2);     // L -> V(0:b, :)
  tile_store(T, c, s, Uinv, b, b, 1);    // U kept in global memory for its inverse
  blk_tsolve(T, c, s, b);
  tile_store(T, c, s, Tout, ldt, b, 1);
#pragma unroll
  for (int r = 0; r < kTE; ++r)
#pragma unroll
    for (int q = 0; q < kTE; ++q) {
      const int i = kTE * c.bi + r, j = kTE * c.bj + q;
      if (i == j && i < b) tau[i] = T.a[r][q];
    }
  if (c.t < b) sgn[c.t] = s.sg[c.t];
  __syncthreads();
  tile_load(T, c, s, Uinv, b, b);  // zeros below the diagonal, identity pad
  __syncthreads();
  blk_inv_upper(T, c, s, b);
  tile_store(T, c, s, Uinv, b, b, 1);
}

// ---------------------------------------------------------------------------
// finalize: write the factored panel in place (v below the diagonal,
// Rh = S (R2 R1) on and above it), for a column panel (rowmajor = 0) or a
// row panel (1).  Rh0 = R2 R1 is full column-major (ld b).
// ---------------------------------------------------------------------------
__global__ void k_panel_finalize(double *P, int64_t ldp, int rowmajor, int m, int b,
                                 const double *V, int64_t ldv, const double *Rh0,
                                 const double *sgn, const int *flag) {
  if (flag[0]) return;
  const int64_t total = (int64_t)m * b;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int r, k;
    if (!rowmajor) {
      r = (int)(idx % m);
      k = (int)(idx / m);
    } else {
      k = (int)(idx % b);
      r = (int)(idx / b);
    }
    const double v = (r > k) ? V[r + (int64_t)k * ldv] : sgn[r] * Rh0[r + (int64_t)k * b];
    if (!rowmajor) P[r + (int64_t)k * ldp] = v;
    else P[k + (int64_t)r * ldp] = v;
  }
}

// Count (per workgroup, at most once) nonzero entries strictly below the
// diagonal of the panel.  A panel with none is already reduced: every column
// has sigma = 0 and the Householder convention gives tau = 0, which the
// reconstruction cannot reproduce, so such panels take the per-column path.
__global__ void k_lower_nonzero(const double *P, int64_t ldp, int rowmajor, int m, int b,
                                int *count) {
  __shared__ int found;
  if (threadIdx.x == 0) found = 0;
  __syncthreads();
  const int64_t total = (int64_t)m * b;
  int mine = 0;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int r, k;
    if (!rowmajor) {
      r = (int)(idx % m);
      k = (int)(idx / m);
    } else {
      k = (int)(idx % b);
      r = (int)(idx / b);
    }
    if (r > k) {
      const double v = rowmajor ? P[k + (int64_t)r * ldp] : P[r + (int64_t)k * ldp];
      if (v != 0.0) mine = 1;
    }
  }
  if (mine) found = 1;
  __syncthreads();
  if (threadIdx.x == 0 && found) atomicAdd(count, 1);
}

int launch_lower_nonzero(const double *P, int64_t ldp, int rowmajor, int m, int b, int *count,
                         hipStream_t s) {
  const int64_t total = (int64_t)m * b;
  int blocks = (int)((total + 1023) / 1024);
  if (blocks > 512) blocks = 512;
  hipLaunchKernelGGL(k_lower_nonzero, dim3(blocks), dim3(256), 0, s, P, ldp, rowmajor, m, b, count);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

int launch_chol_inv(const double *G, int ldg, int b, double rel, double *R, double *Rinv, int *flag,
                    int check_structure, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(kRT), 0, s, G, ldg, b, rel, R, Rinv, flag,
                     check_structure);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

int launch_recon(const double *Qtop, int ldq, int b, double *V, int64_t ldv, double *T, int ldt,
                 double *tau, double *Uinv, double *sgn, const int *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_recon, dim3(1), dim3(kRT), 0, s, Qtop, ldq, b, V, ldv, T, ldt, tau, Uinv,
                     sgn, flag);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

int launch_panel_finalize(double *P, int64_t ldp, int rowmajor, int m, int b, const double *V,
                          int64_t ldv, const double *Rh0, const double *sgn, const int *flag,
                          hipStream_t s) {
  const int64_t total = (int64_t)m * b;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_panel_finalize, dim3(blocks), dim3(256), 0, s, P, ldp, rowmajor, m, b, V,
                     ldv, Rh0, sgn, flag);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace br
