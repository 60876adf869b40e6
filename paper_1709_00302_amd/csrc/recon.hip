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
// factorisations run here in one workgroup of 256 threads.  Each thread keeps
// an 8 x 8 tile of the b x b matrix in registers (16 x 16 tiles cover
// b = 128; sizes below 128 are padded with the identity, which every
// operation below leaves invariant).  The factorisations are blocked by 8:
// the diagonal block (or block row) is handled by its owner thread (or
// owner wave, with shuffles), then the block row / block column is broadcast
// through LDS and every trailing tile takes one rank-8 update, so a block
// step costs one or two workgroup barriers.
//
// Rank-deficient or structurally reduced panels: a pivot of the first
// Cholesky below rel * (original diagonal), or a panel with no nonzero below
// its diagonal, raises a device flag; the remaining kernels of this path then
// return at once and the exact per-column Householder kernel takes the panel.
#include "common.hpp"

namespace br {

constexpr int kRT = 256;  // threads of the register-tiled kernels

struct Tile {
  double a[8][8];
};

struct TileCtx {
  int t, bi, bj, lane;
};

__device__ __forceinline__ TileCtx tile_ctx() {
  TileCtx c;
  c.t = threadIdx.x;
  c.bi = c.t >> 4;
  c.bj = c.t & 15;
  c.lane = c.t & 63;
  return c;
}

// Shared buffers of the blocked steps (double buffered by block parity).
// The block row / column buffers double as the staging area of coalesced
// tile loads and stores (32 columns of 128 rows at a time).
struct Bcast {
  union {
    struct {
      double rb[2][8][kNbMax];  // a block row (8 rows)
      double cb[2][kNbMax][8];  // a block column (8 columns)
    };
    double stage[32 * kNbMax];
  };
  double pb[64];            // a diagonal block
  double d0[kNbMax];        // original diagonal (Cholesky breakdown test)
  double sg[kNbMax];        // LU signs
  int bad;
};

// load a b x b column-major matrix (identity-padded to 128 x 128) through LDS
__device__ __forceinline__ void tile_load(Tile &T, const TileCtx &c, Bcast &s, const double *G,
                                          int ld, int b) {
  for (int ch = 0; ch < 4; ++ch) {
    __syncthreads();
    for (int e = c.t; e < 32 * kNbMax; e += kRT) {
      const int i = e & (kNbMax - 1), j = 32 * ch + (e >> 7);
      s.stage[e] = (i < b && j < b) ? G[i + (int64_t)j * ld] : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    if ((c.bj >> 2) == ch) {
      const int j0 = 8 * (c.bj & 3);
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) T.a[r][q] = s.stage[(j0 + q) * kNbMax + 8 * c.bi + r];
    }
  }
  __syncthreads();
}

// store (parts of) the tile through LDS: mode 0 all, 1 upper (zeros below),
// 2 unit lower (ones on the diagonal, zeros above)
__device__ __forceinline__ void tile_store(const Tile &T, const TileCtx &c, Bcast &s, double *G,
                                           int64_t ld, int b, int mode) {
  for (int ch = 0; ch < 4; ++ch) {
    __syncthreads();
    if ((c.bj >> 2) == ch) {
      const int j0 = 8 * (c.bj & 3);
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int i = 8 * c.bi + r, j = 8 * c.bj + q;
          double v = T.a[r][q];
          if (mode == 1 && j < i) v = 0.0;
          if (mode == 2) v = (i == j) ? 1.0 : (i > j ? v : 0.0);
          s.stage[(j0 + q) * kNbMax + i] = v;
        }
    }
    __syncthreads();
    for (int e = c.t; e < 32 * kNbMax; e += kRT) {
      const int i = e & (kNbMax - 1), j = 32 * ch + (e >> 7);
      if (i < b && j < b) G[i + (int64_t)j * ld] = s.stage[e];
    }
  }
  __syncthreads();
}

// a(r, q) -= sum_l x(r, l) y(l, q) over this thread's tile, x from a block
// column buffer (rows of the tile) and y from a block row buffer.
__device__ __forceinline__ void tile_rank8(Tile &T, const TileCtx &c, const double (*cbuf)[8],
                                           const double (*rbuf)[kNbMax]) {
#pragma unroll
  for (int l = 0; l < 8; ++l) {
    double x[8], y[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) x[r] = cbuf[8 * c.bi + r][l];
#pragma unroll
    for (int q = 0; q < 8; ++q) y[q] = rbuf[l][8 * c.bj + q];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int q = 0; q < 8; ++q) T.a[r][q] -= x[r] * y[q];
  }
}

// Blocked upper Cholesky in place: G = R^T R, R in the upper triangle.
// Block row kb is factored by its 16 owners (one wave) with shuffles; the
// trailing upper tiles then take one rank-8 update.  Returns false (in every
// thread) on a pivot <= rel * d0[k].
__device__ __forceinline__ bool blk_chol(Tile &T, const TileCtx &c, Bcast &s, int b, double rel) {
  if (c.t == 0) s.bad = 0;
  __syncthreads();
  const int nblk = (b + 7) >> 3;
  for (int kb = 0; kb < nblk; ++kb) {
    const int buf = kb & 1;
    if (c.bi == kb && c.bj >= kb) {
      const int dl = (17 * kb) & 63;  // lane of the diagonal tile's owner
      const bool diag = (c.bj == kb);
      bool ok = true;
#pragma unroll
      for (int kr = 0; kr < 8; ++kr) {
        const double d = __shfl(T.a[kr][kr], dl);
        ok = ok && (d > rel * s.d0[8 * kb + kr]);
        const double r = sqrt(d > 0.0 ? d : 1.0), ir = 1.0 / r;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (!diag || q > kr) T.a[kr][q] *= ir;
          else if (q == kr) T.a[kr][q] = r;
        }
#pragma unroll
        for (int k2 = kr + 1; k2 < 8; ++k2) {
          const double f = __shfl(T.a[kr][k2], dl);
#pragma unroll
          for (int q = 0; q < 8; ++q) T.a[k2][q] -= f * T.a[kr][q];
        }
      }
#pragma unroll
      for (int kr = 0; kr < 8; ++kr)
#pragma unroll
        for (int q = 0; q < 8; ++q) s.rb[buf][kr][8 * c.bj + q] = T.a[kr][q];
      if (diag && !ok) s.bad = 1;
    }
    __syncthreads();
    if (s.bad) return false;
    if (c.bi > kb && c.bj >= c.bi) {
#pragma unroll
      for (int l = 0; l < 8; ++l) {
        double x[8], y[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = s.rb[buf][l][8 * c.bi + r];
#pragma unroll
        for (int q = 0; q < 8; ++q) y[q] = s.rb[buf][l][8 * c.bj + q];
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
          for (int q = 0; q < 8; ++q) T.a[r][q] -= x[r] * y[q];
      }
    }
  }
  __syncthreads();
  return true;
}

// Blocked in-place Gauss-Jordan inverse of an upper triangular matrix.
// Pivot block kb: A_kk <- A_kk^-1 (by its owner), A_kj <- A_kk^-1 A_kj,
// A_ij -= A_ik(old) A_kj(new) for i < k < j, A_ik <- -A_ik(old) A_kk^-1.
__device__ __forceinline__ void blk_inv_upper(Tile &T, const TileCtx &c, Bcast &s, int b) {
  const int nblk = (b + 7) >> 3;
  for (int kb = 0; kb < nblk; ++kb) {
    const int buf = kb & 1;
    if (c.bi == kb && c.bj == kb) {
      // in-place inverse of the 8 x 8 upper block, bottom row first
#pragma unroll
      for (int i = 7; i >= 0; --i) {
        const double ii = 1.0 / T.a[i][i];
#pragma unroll
        for (int j = 7; j > i; --j) {
          double acc = 0.0;
#pragma unroll
          for (int l = i + 1; l <= j; ++l) acc += T.a[i][l] * T.a[l][j];
          T.a[i][j] = -acc * ii;
        }
        T.a[i][i] = ii;
#pragma unroll
        for (int j = 0; j < i; ++j) T.a[i][j] = 0.0;
      }
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) s.pb[8 * r + q] = T.a[r][q];
    }
    __syncthreads();
    if (c.bi == kb && c.bj > kb) {  // A_kj <- Pinv A_kj, rows top-down in place
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          double acc = 0.0;
#pragma unroll
          for (int l = r; l < 8; ++l) acc += s.pb[8 * r + l] * T.a[l][q];
          T.a[r][q] = acc;
        }
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) s.rb[buf][r][8 * c.bj + q] = T.a[r][q];
    }
    if (c.bj == kb && c.bi < kb) {  // publish A_ik(old); A_ik <- -A_ik Pinv
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) s.cb[buf][8 * c.bi + r][q] = T.a[r][q];
#pragma unroll
      for (int q = 7; q >= 0; --q)
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          double acc = 0.0;
#pragma unroll
          for (int l = 0; l <= q; ++l) acc += T.a[r][l] * s.pb[8 * l + q];
          T.a[r][q] = -acc;
        }
    }
    __syncthreads();
    if (c.bi < kb && c.bj > kb) tile_rank8(T, c, s.cb[buf], s.rb[buf]);
  }
  __syncthreads();
}

// Blocked LU without pivoting of (W - S), S_k = -sign of the current pivot
// (chosen on the fly).  L (unit, strict lower) and U (upper) overwrite the
// tiles; the signs go to s.sg.
__device__ __forceinline__ void blk_lu_sign(Tile &T, const TileCtx &c, Bcast &s, int b) {
  const int nblk = (b + 7) >> 3;
  for (int kb = 0; kb < nblk; ++kb) {
    const int buf = kb & 1;
    if (c.bi == kb && c.bj == kb) {
#pragma unroll
      for (int kr = 0; kr < 8; ++kr) {
        const double w = T.a[kr][kr];
        const double sgn = (w >= 0.0) ? -1.0 : 1.0;
        const double piv = w - sgn;  // |piv| >= 1
        T.a[kr][kr] = piv;
        s.sg[8 * kb + kr] = sgn;
        const double ip = 1.0 / piv;
#pragma unroll
        for (int i = kr + 1; i < 8; ++i) {
          T.a[i][kr] *= ip;
#pragma unroll
          for (int j = kr + 1; j < 8; ++j) T.a[i][j] -= T.a[i][kr] * T.a[kr][j];
        }
      }
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) s.pb[8 * r + q] = T.a[r][q];
    }
    __syncthreads();
    if (c.bi == kb && c.bj > kb) {  // U_kj = L_kk^-1 A_kj
#pragma unroll
      for (int r = 1; r < 8; ++r)
#pragma unroll
        for (int l = 0; l < r; ++l) {
          const double f = s.pb[8 * r + l];
#pragma unroll
          for (int q = 0; q < 8; ++q) T.a[r][q] -= f * T.a[l][q];
        }
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) s.rb[buf][r][8 * c.bj + q] = T.a[r][q];
    }
    if (c.bj == kb && c.bi > kb) {  // L_ik = A_ik U_kk^-1
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double iu = 1.0 / s.pb[9 * q];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          double v = T.a[r][q];
#pragma unroll
          for (int l = 0; l < q; ++l) v -= T.a[r][l] * s.pb[8 * l + q];
          T.a[r][q] = v * iu;
        }
      }
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) s.cb[buf][8 * c.bi + r][q] = T.a[r][q];
    }
    __syncthreads();
    if (c.bi > kb && c.bj > kb) tile_rank8(T, c, s.cb[buf], s.rb[buf]);
  }
  __syncthreads();
}

// With L (strict lower, unit) and U (upper) in the tiles: T L^T = -U S,
// solved in place over the upper triangle (L is kept), one column block of T
// at a time.
__device__ __forceinline__ void blk_tsolve(Tile &T, const TileCtx &c, Bcast &s, int b) {
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = 8 * c.bi + r, j = 8 * c.bj + q;
      if (j >= i && j < b) T.a[r][q] = -T.a[r][q] * s.sg[j];
    }
  const int nblk = (b + 7) >> 3;
  for (int lb = 0; lb < nblk; ++lb) {
    const int buf = lb & 1;
    if (c.bi == lb && c.bj == lb) {
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) s.pb[8 * r + q] = T.a[r][q];  // L_ll below the diagonal
    }
    __syncthreads();
    if (c.bj == lb) {
      if (c.bi <= lb) {  // T_il = C_il L_ll^-T (upper part only on the diagonal tile)
        const bool diag = (c.bi == lb);
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            if (diag && r > q) continue;
            double v = T.a[r][q];
#pragma unroll
            for (int l = 0; l < q; ++l)
              if (!diag || l >= r) v -= T.a[r][l] * s.pb[8 * q + l];
            T.a[r][q] = v;
          }
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
          for (int q = 0; q < 8; ++q)
            s.cb[buf][8 * c.bi + r][q] = (diag && r > q) ? 0.0 : T.a[r][q];
      } else {  // L_jl below the diagonal block
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
          for (int q = 0; q < 8; ++q) s.cb[buf][8 * c.bi + r][q] = T.a[r][q];
      }
    }
    __syncthreads();
    if (c.bi <= lb && c.bj > lb) {
      // C_ij -= sum_l T(i, l) L(j, l) over the 8 columns l of block lb
#pragma unroll
      for (int l = 0; l < 8; ++l) {
        double x[8], y[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = s.cb[buf][8 * c.bi + r][l];
#pragma unroll
        for (int q = 0; q < 8; ++q) y[q] = s.cb[buf][8 * c.bj + q][l];
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
          for (int q = 0; q < 8; ++q) T.a[r][q] -= x[r] * y[q];
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
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = 8 * c.bi + r, j = 8 * c.bj + q;
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
