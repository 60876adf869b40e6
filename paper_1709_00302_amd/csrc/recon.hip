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
// The O(m b^2) products run on the MFMA GEMM kernel.  The two sequential
// O(b^3) factorisations (Cholesky, LU) run in one workgroup of 1024 threads:
// each thread keeps a 4 x 4 tile of the b x b matrix in registers (32 x 32
// tiles cover b = 128; sizes below 128 are padded with the identity, which
// every operation below leaves invariant; tiles wholly inside the padding are
// neither updated nor stored).  They are blocked by 4 and take one
// workgroup barrier per block step: the diagonal block and its block row are
// handled by the wave that owns them (broadcasts from the diagonal tile's
// lane), the block row and column are published through LDS, and every
// trailing tile takes one rank-4 update.  What other threads need of a
// diagonal block is either fixed in advance or recomputed by each thread from
// the published raw block.  The triangular inverses (R1^-1, R2^-1, U^-1) and
// the solve for T are independent column by column (row by row for T), so they
// run on one workgroup per 16-wide slab with the triangular operand in LDS.
//
// Rank-deficient panels and panels with a structurally zero column: a pivot
// of the first Cholesky below rel * (original diagonal), or a column k whose
// part below the diagonal is exactly zero by the panel's sparsity structure,
// raises a device flag; the remaining kernels of this path then return at once
// and the exact per-column Householder kernel takes the panel.  (For such a
// column the Householder convention sets tau = 0, H = I; the reconstruction
// would return the other valid reflector, tau = 2.)
#include "common.hpp"

namespace br {

constexpr int kRT = 1024;          // threads of the register-tiled kernels
constexpr int kTE = 4;             // tile edge
constexpr int kNTl = kNbMax / kTE;  // tiles per edge (32)
constexpr int kNB4 = kNbMax / kTE;  // 4-wide blocks per edge (32)

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
// tile loads and stores (32 columns of 128 rows at a time, column stride
// kLdStage: with an odd stride the tiles' 4-row pieces of different columns
// fall in different LDS banks).
constexpr int kLdStage = kNbMax + 1;
struct Bcast {
  union {
    struct {
      double rb[2][kTE][kTE][kNTl];  // a block row: rb[.][r][q][J] = row r, column 4 J + q
      double cb[2][kNbMax][kTE];  // a block column (4 columns)
    };
    double stage[32 * kLdStage];
  };
  double pb[2][kTE * kTE];      // the current diagonal block
  double pr[2][kTE];            // reciprocals of its pivots
  double d0[kNbMax];            // original diagonal (Cholesky breakdown test)
  double sg[kNbMax];            // LU signs
  int lz[kNbMax];               // structure check: last nonzero row of each column
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
      const bool in = i < b && j < b;
      const double x = G[in ? i + (int64_t)j * ld : 0];  // clamped: no branch, no wait
      v[ch][k] = in ? x : (i == j ? 1.0 : 0.0);
    }
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int e = c.t + kRT * k;
      s.stage[(e >> 7) * kLdStage + (e & (kNbMax - 1))] = v[ch][k];
    }
    __syncthreads();
    if ((c.bj >> 3) == ch) {
      const int j0 = kTE * (c.bj & 7);
#pragma unroll
      for (int r = 0; r < kTE; ++r)
#pragma unroll
        for (int q = 0; q < kTE; ++q) T.a[r][q] = s.stage[(j0 + q) * kLdStage + kTE * c.bi + r];
    }
  }
  __syncthreads();
}

// store (parts of) the tile: mode 0 all, 1 upper (zeros below), 2 unit lower
// (ones on the diagonal, zeros above).  The tiles are regrouped through LDS 32
// columns at a time so that every global store is a contiguous column run.
__device__ __forceinline__ void tile_store(const Tile &T, const TileCtx &c, Bcast &s, double *G,
                                           int64_t ld, int b, int mode) {
  constexpr int E = 32 * kNbMax / kRT;
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) {
    if (32 * ch >= b) break;
    __syncthreads();
    if ((c.bj >> 3) == ch) {
      const int j0 = kTE * (c.bj & 7);
#pragma unroll
      for (int r = 0; r < kTE; ++r)
#pragma unroll
        for (int q = 0; q < kTE; ++q) {
          const int i = kTE * c.bi + r, j = kTE * c.bj + q;
          double v = T.a[r][q];
          if (mode == 1 && j < i) v = 0.0;
          if (mode == 2) v = (i == j) ? 1.0 : (i > j ? v : 0.0);
          s.stage[(j0 + q) * kLdStage + kTE * c.bi + r] = v;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int e = c.t + kRT * k;
      const int i = e & (kNbMax - 1), j = 32 * ch + (e >> 7);
      if (i < b && j < b) G[i + (int64_t)j * ld] = s.stage[(e >> 7) * kLdStage + i];
    }
  }
  __syncthreads();
}

// The wave that factors block row kb + 1 is on the critical path of step kb:
// it runs at raised priority from the barrier of step kb until it has
// published that row, so that its own trailing update is not slowed down by
// the other waves of its SIMD.
__device__ __forceinline__ void prio_next(const TileCtx &c, int kb) {
  if ((c.t >> 6) == ((kb + 1) >> 1)) __builtin_amdgcn_s_setprio(kPrioCrit);
  else __builtin_amdgcn_s_setprio(kPrioPanel);
}

// Blocked upper Cholesky in place: G = R^T R, R in the upper triangle.  The
// block row kb is factored by its owners (one wave) with the diagonal tile's
// values broadcast from its lane; the trailing upper tiles then take one
// rank-4 update.  Returns false (in every thread) on a pivot <= rel * d0[k]
// (s.d0 holds the original diagonal); the factorisation runs to the end
// either way (a breakdown pivot is replaced by 1) and is checked once.
__device__ __forceinline__ bool blk_chol(Tile &T, const TileCtx &c, Bcast &s, int b, double rel) {
  if (c.t == 0) s.bad = 0;
  __syncthreads();
  const int nblk = (b + kTE - 1) / kTE;
  prio_next(c, -1);
  for (int kb = 0; kb < nblk; ++kb) {
    const int buf = kb & 1;
    if (c.bi == kb && c.bj >= kb && c.bj < nblk) {
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
        for (int q = 0; q < kTE; ++q) s.rb[buf][kr][q][c.bj] = T.a[kr][q];
      if (diag && !ok) s.bad = 1;
    }
    __syncthreads();
    prio_next(c, kb);
    if (c.bi > kb && c.bj >= c.bi && c.bj < nblk) {
#pragma unroll
      for (int l = 0; l < kTE; ++l) {
        double x[kTE], y[kTE];
#pragma unroll
        for (int r = 0; r < kTE; ++r) x[r] = s.rb[buf][l][r][c.bi];
#pragma unroll
        for (int q = 0; q < kTE; ++q) y[q] = s.rb[buf][l][q][c.bj];
#pragma unroll
        for (int r = 0; r < kTE; ++r)
#pragma unroll
          for (int q = 0; q < kTE; ++q) T.a[r][q] -= x[r] * y[q];
      }
    }
  }
  __builtin_amdgcn_s_setprio(kPrioPanel);
  __syncthreads();
  return s.bad == 0;
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

// Blocked LU without pivoting of (W - S), S_k = -sign of the current pivot
// (chosen on the fly).  L (unit, strict lower) and U (upper) overwrite the
// tiles; the signs go to s.sg.  Step kb: the block row (diagonal LU and
// U_kj = L_kk^-1 A_kj) in its wave; the block column publishes its raw
// tiles; after the barrier every thread of a lower block row forms
// L_ik = A_ik U_kk^-1 itself and applies the rank-4 update.
__device__ __forceinline__ void blk_lu_sign(Tile &T, const TileCtx &c, Bcast &s, int b) {
  const int nblk = (b + kTE - 1) / kTE;
  prio_next(c, -1);
  for (int kb = 0; kb < nblk; ++kb) {
    const int buf = kb & 1;
    if (c.bi == kb && c.bj >= kb && c.bj < nblk) {
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
          if (c.lane == dl) {
            s.sg[kTE * kb + kr] = sgn;
            s.pr[buf][kr] = ip;
          }
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
          for (int q = 0; q < kTE; ++q) s.rb[buf][r][q][c.bj] = T.a[r][q];
      }
    }
    if (c.bj == kb && c.bi > kb && c.bi < nblk) {
#pragma unroll
      for (int r = 0; r < kTE; ++r)
#pragma unroll
        for (int q = 0; q < kTE; ++q) s.cb[buf][kTE * c.bi + r][q] = T.a[r][q];
    }
    __syncthreads();
    prio_next(c, kb);
    if (c.bi > kb && c.bj >= kb && c.bi < nblk && c.bj < nblk) {
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
        const double iu = s.pr[buf][q];
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
          for (int q = 0; q < kTE; ++q) y[q] = s.rb[buf][l][q][c.bj];
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

// ---------------------------------------------------------------------------
// kernel A: R = chol(G) (full column-major, zeros below); R^-1 follows in
// k_trinv.  flag[0] is raised on breakdown, and, when `structure` is given
// (the output of k_panel_structure for this panel), if some column k has no
// nonzero strictly below its diagonal once the earlier columns' reflectors are
// applied: that holds exactly when every column j <= k has its last nonzero
// at or above row k (the reflectors of columns 0..k-1 then only mix rows
// 0..k).  For a panel taller than b every column has rows below its diagonal.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRT) void k_chol(const double *G, int ldg, int b, double rel,
                                              double *R, int *flag, const int *structure) {
  __shared__ Bcast s;
  __builtin_amdgcn_s_setprio(kPrioPanel);
  // the flag and structure are read before, and tested after, the matrix
  // loads so that the memory latencies overlap
  const int f0 = flag[0];
  const TileCtx c = tile_ctx();
  int lz = kNbMax;  // columns beyond b never count
  if (structure && c.t < b) lz = structure[kNbMax + c.t] ? kNbMax : structure[c.t];
  Tile T;
  tile_load(T, c, s, G, ldg, b);
  if (f0) return;
  if (structure) {
    if (c.t < kNbMax) s.lz[c.t] = lz;
    __syncthreads();
    if (c.t < 64) {
      // wave 0: lane l holds columns 2l, 2l+1; prefix maximum over columns
      const int k0 = 2 * c.t, k1 = k0 + 1;
      const int p0 = s.lz[k0], p1 = max(p0, s.lz[k1]);
      int inc = p1;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(inc, off);
        if (c.t >= off) inc = max(inc, y);
      }
      int ex = __shfl_up(inc, 1);
      if (c.t == 0) ex = 0;
      const bool zero_col = (k0 < b && max(ex, p0) <= k0) || (k1 < b && max(ex, p1) <= k1);
      const bool any = __any(zero_col);
      if (c.t == 0) s.bad = any ? 1 : 0;
    }
    __syncthreads();
    if (s.bad) {
      if (c.t == 0) flag[0] = 1;
      return;
    }
  }
  if (c.bi == c.bj) {
#pragma unroll
    for (int r = 0; r < kTE; ++r) s.d0[kTE * c.bi + r] = T.a[r][r];  // identity pad beyond b
  }
  if (!blk_chol(T, c, s, b, rel)) {
    if (c.t == 0) flag[0] = 1;
    return;
  }
  tile_store(T, c, s, R, b, b, 1);  // upper factor, zeros below
}

// ---------------------------------------------------------------------------
// kernel B: Qtop (b x b) -> LU with signs: L (unit lower) into V's top block,
// U into a scratch (upper, zeros below), the signs into sgn
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRT) void k_lu(const double *Qtop, int ldq, int b, double *V,
                                            int64_t ldv, double *U, double *sgn, const int *flag) {
  __shared__ Bcast s;
  __builtin_amdgcn_s_setprio(kPrioPanel);
  const int f0 = flag[0];
  const TileCtx c = tile_ctx();
  Tile T;
  tile_load(T, c, s, Qtop, ldq, b);
  if (f0) return;
  blk_lu_sign(T, c, s, b);
  tile_store(T, c, s, V, ldv, b, 2);  // L -> V(0:b, :)
  tile_store(T, c, s, U, b, b, 1);
  if (c.t < b) sgn[c.t] = s.sg[c.t];
}

// ---------------------------------------------------------------------------
// Column- and row-independent triangular solves, one 16-wide slab per
// workgroup of 256 threads (thread t: slab column or row t % 16, the other
// index t / 16 + 16 k for k = 0..7), blocked by 4 with the 4 x 4 diagonal
// pieces fixed in advance; the b x b operand sits in LDS.
// ---------------------------------------------------------------------------
constexpr int kST = 256;           // threads of a slab workgroup
constexpr int kSW = 16;            // slab width
// The triangular operand is kept packed by columns (upper: column j holds
// rows 0..j; strictly lower: rows j+1..127), about half the LDS of the full
// square: at 70 KB a slab workgroup fits on a CU beside one workgroup of the
// large GEMM tiles, so these kernels need not wait for a whole CU to drain
// when they overlap the trailing update.  Reads of the other triangle (made
// for rows whose result is then discarded) stay inside the padded array.
constexpr int kPkPad = 16;
constexpr int kPk = kPkPad + kNbMax * (kNbMax + 1) / 2 + 32;
__device__ __forceinline__ int pk_up(int i, int j) { return kPkPad + j * (j + 1) / 2 + i; }
__device__ __forceinline__ int pk_lo(int i, int j) {
  return kPkPad + j * (2 * kNbMax - j - 1) / 2 + (i - j - 1);
}

struct SlabLds {
  double M[kPk];                   // the triangular operand, packed
  double dg[kNbMax / 4][16];       // inverses of the 4 x 4 diagonal blocks
  double xb[2][4][kSW];            // the current 4-row (or 4-column) block, by parity
};

// M(i, j) = G(i, j) for columns c0 <= j < c1 and all 128 rows, from the
// column-major b x b matrix G; outside b x b (and, for STRICT_LOWER, on and
// above the diagonal) the identity (zero for STRICT_LOWER).  Loads go out in
// batches of kLB per thread before any is written, with clamped addresses
// instead of branches so that nothing waits between them.
template <bool STRICT_LOWER>
__device__ __forceinline__ void slab_load(SlabLds &L, const double *G, int64_t ld, int b, int c0,
                                          int c1) {
  constexpr int kLB = 16;
  // (c1 - c0) is even, so every thread has the same count of elements; the
  // last batch repeats the thread's last element instead of branching
  const int nper = (c1 - c0) * kNbMax / kST;
  for (int u0 = 0; u0 < nper; u0 += kLB) {
    double v[kLB];
#pragma unroll
    for (int u = 0; u < kLB; ++u) {
      const int e = (int)threadIdx.x + kST * min(u0 + u, nper - 1);
      const int i = e & (kNbMax - 1), j = c0 + (e >> 7);
      const bool in = i < b && j < b && (!STRICT_LOWER || i > j);
      v[u] = G[in ? i + (int64_t)j * ld : 0];
    }
#pragma unroll
    for (int u = 0; u < kLB; ++u) {
      const int e = (int)threadIdx.x + kST * min(u0 + u, nper - 1);
      const int i = e & (kNbMax - 1), j = c0 + (e >> 7);
      const bool in = i < b && j < b && (!STRICT_LOWER || i > j);
      if (STRICT_LOWER ? (i > j) : (i <= j))
        L.M[STRICT_LOWER ? pk_lo(i, j) : pk_up(i, j)] =
            in ? v[u] : ((!STRICT_LOWER && i == j) ? 1.0 : 0.0);
    }
  }
}

// M(r, 4 i4 + q), q < 4, for the rows r = g + 16 k with k <= i4 / 4 (the rows
// at or above block i4; others are left untouched).  i4 is a constant after
// unrolling.
__device__ __forceinline__ void slab_fetch_above(const SlabLds &L, int g, int i4,
                                                 double (&m)[8][4]) {
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k <= (i4 >> 2))
#pragma unroll
      for (int q = 0; q < 4; ++q) m[k][q] = L.M[pk_up(g + 16 * k, 4 * i4 + q)];
}

// M(r, 4 j4 + q), q < 4, for the rows r = g + 16 k with k >= j4 / 4.
__device__ __forceinline__ void slab_fetch_below(const SlabLds &L, int g, int j4,
                                                 double (&m)[8][4]) {
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k >= (j4 >> 2))
#pragma unroll
      for (int q = 0; q < 4; ++q) m[k][q] = L.M[pk_lo(g + 16 * k, 4 * j4 + q)];
}

// X = R^-1 for the upper triangular R (columns 16J .. 16J+15 in workgroup J).
__device__ __forceinline__ void slab_trinv(SlabLds &L, const double *R, int ldr, int b, double *X,
                                           int ldx, int J, const int *flag) {
  const int f0 = flag[0];
  const int t = threadIdx.x, cc = t & 15, g = t >> 4;
  const int col = kSW * J + cc;
  const int top = min(b, kSW * J + kSW);  // rows at or above the slab's last column
  const int nb4 = (top + 3) / 4;
  slab_load<false>(L, R, ldr, b, 0, 4 * nb4);  // through the last (padded) 4 x 4 block
  __syncthreads();
  if (f0) return;
  if (t < nb4) {  // inverses of the 4 x 4 diagonal blocks
    double a[kTE][kTE];
#pragma unroll
    for (int r = 0; r < kTE; ++r)
#pragma unroll
      for (int q = 0; q < kTE; ++q) a[r][q] = (q >= r) ? L.M[pk_up(4 * t + r, 4 * t + q)] : 0.0;
    inv4_upper(a);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) L.dg[t][4 * r + q] = a[r][q];
  }
  double B[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) B[k] = (g + 16 * k == col) ? 1.0 : 0.0;
  __syncthreads();
  // Back substitution by 4-row blocks, bottom up, one barrier per block: the
  // owners of the block's rows publish them, every thread then forms the
  // block's solution for its own column (y = D^-1 x) and updates its rows
  // above the block.  The 32 possible steps are unrolled so that every row
  // index is static; steps beyond the slab are skipped (uniformly), and the
  // R entries a step needs are read from LDS before the preceding barrier.
  double mc[8][4], mn[8][4];
#pragma unroll
  for (int i4 = kNB4 - 1; i4 >= 0; --i4) {
    if (i4 < nb4) {
      const int K = i4 >> 2, sub = i4 & 3, par = i4 & 1;
      if (i4 == nb4 - 1) slab_fetch_above(L, g, i4, mc);
      const bool own = (g >> 2) == sub;
      if (own) L.xb[par][g & 3][cc] = B[K];
      if (i4 > 0) slab_fetch_above(L, g, i4 - 1, mn);
      __syncthreads();
      double xv[4], y[4];
#pragma unroll
      for (int l = 0; l < 4; ++l) xv[l] = L.xb[par][l][cc];
      const double *P = L.dg[i4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double acc = 0.0;
#pragma unroll
        for (int l = q; l < 4; ++l) acc += P[4 * q + l] * xv[l];
        y[q] = acc;
      }
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) B[k] -= mc[k][q] * y[q];
      double u = B[K];
#pragma unroll
      for (int q = 0; q < 4; ++q) u -= mc[K][q] * y[q];
      const int gl = g & 3;
      const double yo = gl == 0 ? y[0] : gl == 1 ? y[1] : gl == 2 ? y[2] : y[3];
      B[K] = own ? yo : ((g >> 2) < sub ? u : B[K]);
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) mc[k][q] = mn[k][q];
    }
  }
  if (col < b) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = g + 16 * k;
      if (r < b) X[r + (int64_t)col * ldx] = B[k];
    }
  }
}

// T L^T = C with C = -U S (U upper, S = diag(sgn)), L unit lower (strict
// part in V's top block): rows 16I .. 16I+15 of T in workgroup I, solved by
// 4-column blocks left to right.  T is upper triangular; tau = diag(T).
__device__ __forceinline__ void slab_tsolve(SlabLds &L, const double *U, const double *Vt,
                                            int64_t ldv, const double *sgn, int b, double *Tout,
                                            int ldt, double *tau, int I, const int *flag) {
  const int f0 = flag[0];
  const int t = threadIdx.x, rr = t & 15, g = t >> 4;
  const int row = kSW * I + rr;
  const int nb4 = (b + 3) / 4;
  // L(j, l) for l < j, packed by columns; only columns l >= 16 I
  // (and rows below them) take part in this slab's solve
  double Cv[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int j = g + 16 * k;
    const bool in = row < b && j < b && j >= row;
    const double u = U[in ? row + (int64_t)j * b : 0], sj = sgn[in ? j : 0];
    Cv[k] = in ? -u * sj : 0.0;
  }
  slab_load<true>(L, Vt, ldv, b, kSW * I, 4 * nb4);
  __syncthreads();
  if (f0) return;
  // forward by 4-column blocks, one barrier per block, unrolled like the
  // back substitution of slab_trinv (steps outside the slab skipped
  // uniformly, the L entries below the block read before the barrier)
  const int j0 = (kSW * I) / 4;
  double mc[8][4], mn[8][4];
#pragma unroll
  for (int j4 = 0; j4 < kNB4; ++j4) {
    if (j4 >= j0 && j4 < nb4) {
      const int K = j4 >> 2, sub = j4 & 3, par = j4 & 1;
      if (j4 == j0) slab_fetch_below(L, g, j4, mc);
      const bool own = (g >> 2) == sub;
      if (own) L.xb[par][g & 3][rr] = Cv[K];
      if (j4 + 1 < kNB4) slab_fetch_below(L, g, j4 + 1, mn);
      __syncthreads();
      // the block's 4 columns of this row: forward substitution with the unit
      // lower diagonal block of L (every thread, for its own row)
      double y[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double v = L.xb[par][q][rr];
#pragma unroll
        for (int l = 0; l < q; ++l) v -= y[l] * L.M[pk_lo(4 * j4 + q, 4 * j4 + l)];
        y[q] = v;
      }
#pragma unroll
      for (int k = K + 1; k < 8; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) Cv[k] -= y[q] * mc[k][q];
      double u = Cv[K];
#pragma unroll
      for (int q = 0; q < 4; ++q) u -= y[q] * mc[K][q];
      const int gl = g & 3;
      const double yo = gl == 0 ? y[0] : gl == 1 ? y[1] : gl == 2 ? y[2] : y[3];
      Cv[K] = own ? yo : ((g >> 2) > sub ? u : Cv[K]);
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) mc[k][q] = mn[k][q];
    }
  }
  if (row < b) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int j = g + 16 * k;
      if (j < b) {
        const double v = (j >= row) ? Cv[k] : 0.0;
        Tout[row + (int64_t)j * ldt] = v;
        if (j == row) tau[row] = v;
      }
    }
  }
}

__global__ __launch_bounds__(kST) void k_trinv(const double *R, int ldr, int b, double *X, int ldx,
                                               const int *flag) {
  __shared__ SlabLds L;
  __builtin_amdgcn_s_setprio(kPrioPanel);
  slab_trinv(L, R, ldr, b, X, ldx, blockIdx.x, flag);
}

// workgroups 0 .. ns-1: rows of T; ns .. 2ns-1: columns of U^-1
__global__ __launch_bounds__(kST) void k_recon_solve(const double *U, const double *V, int64_t ldv,
                                                     const double *sgn, int b, double *Tout,
                                                     int ldt, double *tau, double *Uinv,
                                                     const int *flag) {
  __shared__ SlabLds L;
  __builtin_amdgcn_s_setprio(kPrioPanel);
  const int ns = (b + kSW - 1) / kSW;
  if ((int)blockIdx.x < ns)
    slab_tsolve(L, U, V, ldv, sgn, b, Tout, ldt, tau, blockIdx.x, flag);
  else
    slab_trinv(L, U, b, b, Uinv, b, blockIdx.x - ns, flag);
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
  __builtin_amdgcn_s_setprio(kPrioPanel);
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

// Sparsity structure of the m x b panel below its diagonal, for the check of
// k_chol: structure[k] = the last row r < b with r > k and P(r, k) != 0 (0 if
// none), structure[kNbMax + k] = 1 when column k has a nonzero in some row
// >= b.  Both zero on entry; every workgroup reduces its share in LDS and then
// raises the global entries (atomic maximum for the rows, plain stores of one
// value for the flags).  The loads are issued four at a time.
__global__ void k_panel_structure(const double *P, int64_t ldp, int rowmajor, int m, int b,
                                  int *structure) {
  __shared__ int s_top[kNbMax], s_deep[kNbMax];
  __builtin_amdgcn_s_setprio(kPrioPanel);
  const int t = threadIdx.x;
  for (int k = t; k < kNbMax; k += blockDim.x) {
    s_top[k] = 0;
    s_deep[k] = 0;
  }
  __syncthreads();
  const int64_t total = (int64_t)m * b;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  constexpr int U = 4;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x + t; base < total; base += U * stride) {
    double v[U];
    int r[U], k[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t idx = base + u * stride;
      const int64_t ic = idx < total ? idx : 0;  // clamped: the value is ignored
      if (!rowmajor) {
        r[u] = (int)(ic % m);
        k[u] = (int)(ic / m);
      } else {
        k[u] = (int)(ic % b);
        r[u] = (int)(ic / b);
      }
      v[u] = rowmajor ? P[k[u] + (int64_t)r[u] * ldp] : P[r[u] + (int64_t)k[u] * ldp];
      if (idx >= total) v[u] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (v[u] != 0.0 && r[u] > k[u]) {
        if (r[u] >= b) s_deep[k[u]] = 1;
        else atomicMax(&s_top[k[u]], r[u]);
      }
    }
  }
  __syncthreads();
  for (int k = t; k < b; k += blockDim.x) {
    if (s_top[k] > 0) atomicMax(&structure[k], s_top[k]);
    if (s_deep[k]) structure[kNbMax + k] = 1;
  }
}

int launch_panel_structure(const double *P, int64_t ldp, int rowmajor, int m, int b,
                           int *structure, hipStream_t s) {
  const int64_t total = (int64_t)m * b;
  int blocks = (int)((total + 1023) / 1024);
  if (blocks > 512) blocks = 512;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_panel_structure, dim3(blocks), dim3(256), 0, s, P, ldp, rowmajor, m, b,
                     structure);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

int launch_chol_inv(const double *G, int ldg, int b, double rel, double *R, double *Rinv, int *flag,
                    const int *structure, hipStream_t s) {
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(kRT), 0, s, G, ldg, b, rel, R, flag, structure);
  BR_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_trinv, dim3((b + kSW - 1) / kSW), dim3(kST), 0, s, R, b, b, Rinv, b,
                     (const int *)flag);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

int launch_recon(const double *Qtop, int ldq, int b, double *V, int64_t ldv, double *T, int ldt,
                 double *tau, double *Uinv, double *sgn, double *Uscr, const int *flag,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_lu, dim3(1), dim3(kRT), 0, s, Qtop, ldq, b, V, ldv, Uscr, sgn, flag);
  BR_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_recon_solve, dim3(2 * ((b + kSW - 1) / kSW)), dim3(kST), 0, s,
                     (const double *)Uscr, (const double *)V, ldv, (const double *)sgn, b, T, ldt,
                     tau, Uinv, flag);
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
