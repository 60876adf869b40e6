// ozaki.hip -- the exact-split form of the trailing-update products (gfx950).
//
// Not in the paper (which is FP64 only): a product C = op(A) op(B) whose
// operands are split into int8 slices and multiplied on the int8 matrix
// cores, where products accumulate exactly in int32 (the error-free slicing
// of Ozaki, Ogita, Oishi and Rump, on integer units).
//
// The inner dimension is cut into one or two segments (the rank-2k updates
// take [W | V] [V | W]^T as two: their halves differ in scale by the norm of
// the matrix).  In segment s, row i of op(A) is scaled by 2^-e_si so that its
// entries are below (127/128)/2 in magnitude, rounded to a multiple of 2^-56
// (remainder at most 2^-57) and written as kOzS = 7 signed base-256 digits:
//     a 2^-e_si = sum_{p=1..7} d_p 256^-p + r,   d_p in [-128, 127], |r| <= 2^-57
// (the integer a 2^(56 - e_si) cut into bytes from the least significant up,
// each byte taken in [-128, 127] with a carry into the next: every step is
// exact in FP64, and the bound on the entries keeps the top digit within
// [-127, 127]); column j of op(B) likewise with 2^-f_sj.  Then
//     C_ij = sum_s 2^(e_si + f_sj) sum_t 256^-t sum_{p+q=t} sum_{k in s} d^A_p(i,k) d^B_q(k,j),
// keeping the 28 pairs with p + q <= 8.  Pairs of equal t share one int32
// accumulator, which the kernel folds into FP64 at the end of a segment and
// every kOzKF terms of k (at most 7 x 2048 x 128^2 < 2^31 in magnitude, so
// the int32 sums are exact).  Per term of k the dropped pairs (6 of order 9,
// each below 2^-58, and fewer of higher order) and the two rounding
// remainders (together at most 2^-57, the scaled entries being below 1/2)
// add up to less than 2^-54 of 2^(e_si + f_sj), and 2^e_si is at most
// 4 (128/127) times the largest entry of the row in the segment: the error of
// C_ij is below 2^-49 sum_s K_s max_k|a_ik| max_k|b_kj|, under the worst-case
// bound of an FP64 dot product of length K.
//
// Slices are stored as planes: plane p of op(A) holds M rows of Kp int8
// (each segment zero padded to a multiple of 64, Kp the sum), plane q of
// op(B) N rows likewise, in 64 x 64 blocks (below).  The product kernel
// copies the blocks of every plane into LDS; a lane's 16 bytes of an MFMA
// operand are one LDS read.
// v_mfma_i32_16x16x64_i8 (measured on gfx950): lane l supplies A(l % 16,
// 16 (l / 16) + e) and B(16 (l / 16) + e, l % 16) as bytes e = 0..15 and
// receives D(4 (l / 16) + e, l % 16) in element e.
#include "common.hpp"

namespace br {

typedef int v4i __attribute__((ext_vector_type(4)));

// The planes are stored in 64 x 64 blocks: block (rb, kb) of plane p (rows
// 64 rb .., plane columns 64 kb ..) is the 4 KB at ((rb nKB + kb) kOzS + p)
// kOzBlk, nKB = Kp / 64, holding row r's 16-byte chunk c at oz_swz(r, c):
// 64 r + 16 (c ^ ((r / 4) mod 4)).  That is also the block's image in the
// product kernel's LDS (a straight copy), where the 16 rows one MFMA operand
// read touches fall on distinct banks.  Rows are padded to a multiple of 64.
__device__ __forceinline__ int oz_swz(int r, int c) { return r * 64 + ((c ^ ((r >> 2) & 3)) << 4); }
constexpr int kOzBlk = 64 * 64;             // bytes of one plane's block
constexpr int kOzStage = 2 * kOzS * kOzBlk; // both operands, all planes

// Operand x of a product as rows: row r, entry k is op(A)(r, k) (isB = 0) or
// op(B)(k, r) (isB = 1).  The symmetric pattern reads the lower triangle
// (entry (r, k) with r < k at (k, r)) and the rotated one shifts k by rot
// modulo K.  Segment 0 is k < ks (all of K when ks = K), segment 1 the rest;
// in the planes segment 0 takes columns [0, L0) and segment 1 [L0, Kp).
struct OzSrc {
  const double *X;
  int64_t ld;
  int op, isB, rows, K, rot;
  int ks, L0, Kp;
};
__device__ __forceinline__ bool oz_row_contig(const OzSrc &s) {
  return s.isB ? (s.op != B_N) : (s.op != A_T);  // A_N, A_SYM, B_T, B_TROT
}
__device__ __forceinline__ double oz_at(const OzSrc &s, int r, int k) {
  if (!s.isB) {
    if (s.op == A_N) return s.X[r + (int64_t)k * s.ld];
    if (s.op == A_T) return s.X[k + (int64_t)r * s.ld];
    return (r >= k) ? s.X[r + (int64_t)k * s.ld] : s.X[k + (int64_t)r * s.ld];
  }
  if (s.op == B_N) return s.X[k + (int64_t)r * s.ld];
  if (s.op == B_T) return s.X[r + (int64_t)k * s.ld];
  int kr = k + s.rot;
  if (kr >= s.K) kr -= s.K;
  return s.X[r + (int64_t)kr * s.ld];
}

// segment of plane block kb (64 columns) and the operand range it maps to
__device__ __forceinline__ void oz_block(const OzSrc &s, int kb, int *seg, int *k0, int *klim) {
  const int c = kb * 64;
  if (c < s.L0) {
    *seg = 0; *k0 = c; *klim = s.ks;
  } else {
    *seg = 1; *k0 = s.ks + (c - s.L0); *klim = s.K;
  }
}

// Stage the 64 x 64 block (rows r0.., entries k0.. below klim) into t[r][k]
// with loads that follow the contiguous dimension; other entries are 0.
// All 16 loads of a thread are issued before its first LDS store.
__device__ __forceinline__ void oz_stage(const OzSrc &s, int r0, int k0, int klim,
                                         double (*t)[65]) {
  const int tid = threadIdx.x;
  const bool rc = oz_row_contig(s);
  double v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int a = tid & 63, c = (tid >> 6) + 4 * i;
    const int rl = rc ? a : c, kl = rc ? c : a;
    const int r = r0 + rl, k = k0 + kl;
    v[i] = (r < s.rows && k < klim) ? oz_at(s, r, k) : 0.0;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int a = tid & 63, c = (tid >> 6) + 4 * i;
    const int rl = rc ? a : c, kl = rc ? c : a;
    t[rl][kl] = v[i];
  }
}

// |x| for a finite x, +Inf for NaN and +-Inf (fmax would skip a NaN): a row
// or column with a non-finite entry gets the exponent kOzNonFinite, and every
// result it meets is NaN, as in FP64 arithmetic.
constexpr int kOzNonFinite = 1 << 20;
__device__ __forceinline__ double oz_mag(double x) {
  const double a = fabs(x);
  return a <= 1.7976931348623157e308 ? a : __builtin_inf();
}

// largest |entry| of each row in each segment (rmax[seg rows + r]), as the
// bits of a non-negative double (atomicMax on them orders like the values);
// rmax is zero at launch.  A symmetric operand (one segment) visits the lower
// blocks only and credits each entry to both its row and its column.
__global__ __launch_bounds__(256) void k_oz_rowmax(OzSrc s, unsigned long long *rmax) {
  const int kb = blockIdx.x, rb = blockIdx.y;
  const bool sym = !s.isB && s.op == A_SYM;
  if (sym && rb < kb) return;
  int seg, k0, klim;
  oz_block(s, kb, &seg, &k0, &klim);
  __shared__ double t[64][65];
  oz_stage(s, rb * 64, k0, klim, t);
  __syncthreads();
  // four adjacent lanes per row (per column): a quarter each, then combined
  const int tid = threadIdx.x, x = tid >> 2, q = tid & 3;
  unsigned long long *rm = rmax + (int64_t)seg * s.rows;
  double m = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) m = fmax(m, oz_mag(t[x][16 * q + k]));
  m = fmax(m, __shfl_xor(m, 1));
  m = fmax(m, __shfl_xor(m, 2));
  const int r = rb * 64 + x;
  if (q == 0 && r < s.rows && m > 0.0)
    atomicMax(rm + r, (unsigned long long)__double_as_longlong(m));
  if (sym && rb > kb) {  // column maxima (the mirrored rows)
    double c = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) c = fmax(c, oz_mag(t[16 * q + i][x]));
    c = fmax(c, __shfl_xor(c, 1));
    c = fmax(c, __shfl_xor(c, 2));
    const int rr = kb * 64 + x;
    if (q == 0 && rr < s.rows && c > 0.0)
      atomicMax(rm + rr, (unsigned long long)__double_as_longlong(c));
  }
}

// exponent e of a row: its entries are below (127/128) 2^(e - 1) in
// magnitude (0 for a zero row)
__global__ void k_oz_exps(const unsigned long long *rmax, int count, int *ex) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= count) return;
  const double m = __longlong_as_double((long long)rmax[r]);
  int e = 0;
  if (!(m <= 1.7976931348623157e308)) {
    e = kOzNonFinite;
  } else if (m > 0.0) {
    const double f = frexp(m, &e);  // m = f 2^e, f in [0.5, 1)
    if (f >= 127.0 / 128.0) ++e;    // then m < (127/128) 2^e
    ++e;
  }
  ex[r] = e;
}

// The digits of 4 consecutive entries of one row, packed 4 to a word per
// plane.  With Y = rint(a 2^(56 - e)) (|Y| < 127 2^48) and C the integer with
// seven bytes 0x80, Z = Y + C lies in [0, 2^56); byte k of Z less 128 is the
// digit of weight 256^k (that subtraction makes the carries: Y = Z - C), and
// as an int8 it is the byte with its top bit flipped.  Y is assembled from
// two exact 32-bit conversions.
__device__ __forceinline__ void oz_digits4(const double *v, int e, unsigned *w) {
  unsigned zl[4], zh[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double r = (e == kOzNonFinite) ? 0.0 : rint(ldexp(v[c], 56 - e));
    const double h = floor(r * 0x1p-32);
    const double l = fma(-h, 0x1p32, r);  // exact, in [0, 2^32)
    const uint64_t Y = ((uint64_t)(int64_t)(int)h << 32) + (uint64_t)(unsigned)l;
    const uint64_t Z = Y + 0x0080808080808080ull;
    zl[c] = (unsigned)Z;
    zh[c] = (unsigned)(Z >> 32);
  }
#pragma unroll
  for (int p = 0; p < kOzS; ++p) {  // plane p holds the digit of weight 256^(6 - p)
    const int k = kOzS - 1 - p;
    unsigned x = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const unsigned src = k < 4 ? zl[c] : zh[c];
      x |= ((src >> (8 * (k & 3))) & 0xffu) << (8 * c);
    }
    w[p] = x ^ 0x80808080u;
  }
}

// The digit planes of the operand (blocked as above; zero in the padding).
// Thread t writes bytes 16 t .. 16 t + 15 of every plane's block: row t / 4,
// chunk (t % 4) ^ ((t / 16) % 4), 16 entries.  A symmetric operand stages
// its lower blocks only and writes each one twice (as rows and, mirrored, as
// columns).
__global__ __launch_bounds__(256) void k_oz_slice(OzSrc s, const int *ex, int8_t *planes) {
  const int kb = blockIdx.x, rb = blockIdx.y;
  const bool sym = !s.isB && s.op == A_SYM;
  if (sym && rb < kb) return;
  int seg, k0, klim;
  oz_block(s, kb, &seg, &k0, &klim);
  __shared__ double t[64][65];
  oz_stage(s, rb * 64, k0, klim, t);
  __syncthreads();
  const int nKB = s.Kp / 64;
  const int *exs = ex + (int64_t)seg * s.rows;
  const int tid = threadIdx.x, rl = tid >> 2, c = (tid & 3) ^ ((rl >> 2) & 3);
  const int passes = (sym && rb > kb) ? 2 : 1;
  for (int pass = 0; pass < passes; ++pass) {
    const int RB = pass ? kb : rb, KB = pass ? rb : kb;
    const int r = RB * 64 + rl;
    const int e = r < s.rows ? exs[r] : 0;
    unsigned w[4][kOzS];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      double v[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int kl = 16 * c + 4 * g + x;
        v[x] = pass ? t[kl][rl] : t[rl][kl];
      }
      oz_digits4(v, e, w[g]);
    }
    int8_t *dst = planes + ((int64_t)RB * nKB + KB) * kOzS * kOzBlk + 16 * tid;
#pragma unroll
    for (int p = 0; p < kOzS; ++p)
      *(v4i *)(dst + p * kOzBlk) = v4i{(int)w[0][p], (int)w[1][p], (int)w[2][p], (int)w[3][p]};
  }
}

struct OzDesc {
  const int8_t *PA, *PB;   // blocked planes of op(A) (M rows) and op(B) (N rows)
  const int *ea, *eb;      // exponents: ea[seg M + row], eb[seg N + col]
  int M, N, Kp, L0;        // plane columns, and where segment 1 starts
  int kchunk;              // k range of one k chunk (multiple of 64)
  double *C;
  int64_t ldc;
  double alpha, beta;
  double *part;            // split-k partials (E_PART)
  int c0, c1;              // SYR2K column range
  unsigned long long *rec; // SYR2K: row / column maxima of the result (or null) ...
  int rec_off;             // ... for indices >= rec_off, stored at index - rec_off
  int nI, nJ, nZ;          // tiles: row blocks, column blocks, k chunks
  const int *abort;
};

// 64 x 64 output tile, 4 waves as 2 x 2 (32 x 32 each: 2 x 2 blocks of 16 x 16).
// One LDS stage buffer (56 KB) and at most 256 registers per lane, so that
// two workgroups share a CU and hide each other's stage loads, per-tile
// prologue and C round trip (measured on SY2SB n=16384 against a
// double-buffered ring with one workgroup per CU: SYR2K products 99.6 ->
// 81.6 ms, SYMM products about 59 -> 52 ms).
template <int EPI>
__global__ __launch_bounds__(256, 2) void k_gemm_oz(OzDesc d) {
  __shared__ __attribute__((aligned(16))) int8_t lds[kOzStage];
  if (d.abort && *d.abort != 0) return;
  // one tile per workgroup: the SYR2K enumerates only the tiles that reach
  // the lower triangle (column J holds row blocks J .. nI-1), the others
  // every (row block, column block, k chunk) with the row block fastest
  const int T = blockIdx.x;
  int i0, j0, kbeg, kend, z = 0;
  int ib, jb;  // the tile's 64-row blocks in the planes of op(A) and op(B)
  if (EPI == E_SYR2K) {
    // J: the largest column with S(J) = J nI - J (J - 1) / 2 <= T
    const double b2 = d.nI + 0.5;
    int J = (int)(b2 - sqrt(b2 * b2 - 2.0 * T));
    J = max(0, min(J, d.nJ - 1));
    auto S = [&](int x) { return x * d.nI - x * (x - 1) / 2; };
    while (J > 0 && S(J) > T) --J;
    while (J + 1 < d.nJ && S(J + 1) <= T) ++J;
    const int I = J + (T - S(J));
    i0 = d.c0 + I * 64;
    j0 = d.c0 + J * 64;
    ib = I;  // (the planes start at row c0)
    jb = J;
    kbeg = 0;
    kend = d.Kp;
  } else {
    const int I = T % d.nI, J = (T / d.nI) % d.nJ;
    z = T / (d.nI * d.nJ);
    i0 = I * 64;
    j0 = J * 64;
    ib = I;
    jb = J;
    kbeg = z * d.kchunk;
    kend = min(d.Kp, kbeg + d.kchunk);
  }
  const int Nlim = (EPI == E_SYR2K) ? d.c1 : d.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  // staging, global -> LDS without registers: the blocks are stored as their
  // LDS image, so wave w copies bytes 1024 w .. 1024 w + 1023 of every
  // plane's block of both operands, one 16-byte piece per lane (written
  // lane-contiguously by the instruction)
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  typedef __attribute__((address_space(1))) const void gvoid;
  typedef __attribute__((address_space(3))) void lvoid;
  const int64_t rowblk = (int64_t)(d.Kp / 64) * kOzS * kOzBlk;  // one 64-row block, all planes
  const int8_t *gA = d.PA + (int64_t)ib * rowblk + wv * 1024 + 16 * lane;
  const int8_t *gB = d.PB + (int64_t)jb * rowblk + wv * 1024 + 16 * lane;
  auto issue_stage = [&](int k0) {
    int8_t *base = lds + wv * 1024;
    const int64_t kofs = (int64_t)(k0 / 64) * kOzS * kOzBlk;
#pragma unroll
    for (int p = 0; p < kOzS; ++p) {
      __builtin_amdgcn_global_load_lds((gvoid *)(gA + kofs + p * kOzBlk), (lvoid *)(base + p * kOzBlk),
                                       16, 0, 0);
      __builtin_amdgcn_global_load_lds((gvoid *)(gB + kofs + p * kOzBlk),
                                       (lvoid *)(base + (kOzS + p) * kOzBlk), 16, 0, 0);
    }
  };
  // the lane's operand rows in the block, and its result rows / columns
  int fa[2], fb[2], er[2][4], ec[2];
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    fa[f] = oz_swz(wm * 32 + f * 16 + (lane & 15), lane >> 4);
    fb[f] = oz_swz(wn * 32 + f * 16 + (lane & 15), lane >> 4);
    ec[f] = min(j0 + wn * 32 + f * 16 + (lane & 15), d.N - 1);
#pragma unroll
    for (int e = 0; e < 4; ++e) er[f][e] = min(i0 + wm * 32 + f * 16 + 4 * (lane >> 4) + e, d.M - 1);
  }
  double acc64[2][2][4];
  v4i acc[kOzS][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
      for (int e = 0; e < 4; ++e) acc64[a][b][e] = 0.0;
#pragma unroll
      for (int t = 0; t < kOzS; ++t) acc[t][a][b] = v4i{0, 0, 0, 0};
    }
  // int32 sums -> FP64, scaled by the segment's row and column exponents
  auto fold = [&](int seg) {
    const int *ea = d.ea + (int64_t)seg * d.M, *eb = d.eb + (int64_t)seg * d.N;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int xb = eb[ec[b]];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          double s = 0.0;
#pragma unroll
          for (int t = kOzS - 1; t >= 0; --t)  // pair order t + 2, smallest first
            s += (double)acc[t][a][b][e] * ldexp(1.0, -8 * (t + 2));
          const int x = ea[er[a][e]] + xb;
          acc64[a][b][e] += (x >= kOzNonFinite / 2) ? __builtin_nan("") : ldexp(s, x);
        }
#pragma unroll
        for (int t = 0; t < kOzS; ++t) acc[t][a][b] = v4i{0, 0, 0, 0};
      }
  };
  const int nst = (kend - kbeg) / 64;
  if (nst > 0) {
    issue_stage(kbeg);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  }
  // runs of stages between folds: a run ends at the end of a segment or
  // after kOzKF terms of k
  int st = 0;
  while (st < nst) {
    const int k0 = kbeg + 64 * st;
    const int seg = k0 >= d.L0 ? 1 : 0;
    int stop = min(nst, st + kOzKF / 64);
    if (seg == 0) stop = min(stop, (d.L0 - kbeg) / 64);
    for (; st < stop; ++st) {
      const int8_t *A = lds, *B = A + kOzS * kOzBlk;
      if (st > 0) {
        // this stage into the buffer (its readers passed the barrier that
        // ended the previous stage)
        issue_stage(kbeg + 64 * st);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
      }
      v4i bq[kOzS][2];
#pragma unroll
      for (int q = 0; q < kOzS; ++q)
#pragma unroll
        for (int f = 0; f < 2; ++f) bq[q][f] = *(const v4i *)(B + q * kOzBlk + fb[f]);
#pragma unroll
      for (int p = 0; p < kOzS; ++p) {
        v4i ap[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) ap[f] = *(const v4i *)(A + p * kOzBlk + fa[f]);
#pragma unroll
        for (int q = 0; q + p < kOzS; ++q)  // pairs with (p+1) + (q+1) <= 8
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
              acc[p + q][a][b] =
                  __builtin_amdgcn_mfma_i32_16x16x64_i8(ap[a], bq[q][b], acc[p + q][a][b], 0, 0, 0);
      }
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }
    fold(seg);
  }
  // element e of block (a, b) is row 4 (lane / 16) + e, column lane % 16.
  // SYR2K with d.rec: the largest |new value| of every row and every column
  // with index >= d.rec_off (a trailing block of the symmetric matrix, whose
  // row maxima are those of its stored rows and columns) goes to
  // d.rec[index - rec_off], one atomicMax per row / column and wave.
  double rowm[2][4], colm[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    colm[a] = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) rowm[a][e] = 0.0;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = i0 + wm * 32 + a * 16 + 4 * (lane >> 4) + e;
        const int col = j0 + wn * 32 + b * 16 + (lane & 15);
        bool in = row < d.M && col < Nlim;
        if (EPI == E_SYR2K) in = in && row >= col;
        if (!in) continue;
        const double v = acc64[a][b][e];
        if (EPI == E_AXPBY) {
          double *c = d.C + row + (int64_t)col * d.ldc;
          *c = (d.beta == 0.0) ? d.alpha * v : d.alpha * v + d.beta * (*c);
        } else if (EPI == E_PART) {
          d.part[(int64_t)z * d.M * d.N + row + (int64_t)col * d.M] = v;
        } else {
          double *c = d.C + row + (int64_t)col * d.ldc;
          const double x = *c - v;
          *c = x;
          if (col >= d.rec_off) {
            rowm[a][e] = fmax(rowm[a][e], oz_mag(x));
            colm[b] = fmax(colm[b], oz_mag(x));
          }
        }
      }
  if (EPI == E_SYR2K && d.rec) {
    // the tile's row and column maxima: over the lanes of a wave by
    // shuffles, over the two waves sharing a row (column) block in LDS, then
    // one atomicMax per row and column of the tile
    __syncthreads();  // every wave is done with the stage buffer
    double *rmx = (double *)lds, *cmx = rmx + 2 * 64;  // [2 waves][64]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int e = 0; e < 4; ++e) {  // the 16 lanes of one row: lane % 16 varies
        double m = rowm[a][e];
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) m = fmax(m, __shfl_xor(m, off));
        if ((lane & 15) == 0) rmx[wn * 64 + wm * 32 + a * 16 + 4 * (lane >> 4) + e] = m;
      }
#pragma unroll
    for (int b = 0; b < 2; ++b) {  // the 4 lanes of one column: lane / 16 varies
      double m = colm[b];
      m = fmax(m, __shfl_xor(m, 16));
      m = fmax(m, __shfl_xor(m, 32));
      if ((lane >> 4) == 0) cmx[wm * 64 + wn * 32 + b * 16 + (lane & 15)] = m;
    }
    __syncthreads();
    const int tid = threadIdx.x;
    if (tid < 128) {
      const int x = tid & 63;
      const double m = (tid < 64) ? fmax(rmx[x], rmx[64 + x]) : fmax(cmx[x], cmx[64 + x]);
      const int idx = ((tid < 64) ? i0 : j0) + x;
      if (m > 0.0 && idx >= d.rec_off)
        atomicMax(d.rec + (idx - d.rec_off), (unsigned long long)__double_as_longlong(m));
    }
  }
}

int oz_plane_cols(int K, int ks, int *L0) {
  if (ks <= 0 || ks >= K) ks = K;
  *L0 = (ks + 63) / 64 * 64;
  return *L0 + (K - ks + 63) / 64 * 64;
}

int oz_slice(const double *X, int64_t ld, int op, int rows, int K, int ks, int rot, int isB,
             unsigned long long *rmax, int *ex, int8_t *planes, hipStream_t s,
             const unsigned long long *rmax_in) {
  if (rows <= 0) return 0;
  if (ks <= 0 || ks >= K) ks = K;
  int L0 = 0;
  const int Kp = oz_plane_cols(K, ks, &L0);
  if (op == A_SYM && !isB && ks != K) return BANDRED_ERR_UNSUPPORTED;
  OzSrc src{X, ld, op, isB, rows, K, rot, ks, L0, Kp};
  const int nseg = (ks < K) ? 2 : 1;
  if (rmax_in && nseg != 1) return BANDRED_ERR_UNSUPPORTED;
  const dim3 grid(Kp / 64, (rows + 63) / 64);
  if (rmax_in) {
    rmax = const_cast<unsigned long long *>(rmax_in);  // (read only below)
  } else {
    int rc = launch_fill_u32((unsigned *)rmax, 2 * (int64_t)nseg * rows, 0u, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_oz_rowmax, grid, dim3(256), 0, s, src, rmax);
    BR_HIP_CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_oz_exps, dim3((nseg * rows + 255) / 256), dim3(256), 0, s,
                     (const unsigned long long *)rmax, nseg * rows, ex);
  BR_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_oz_slice, grid, dim3(256), 0, s, src, (const int *)ex, planes);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

int oz_gemm(int epi, const int8_t *PA, const int8_t *PB, const int *ea, const int *eb, int M,
            int N, int Kp, int L0, int ksplit, int kchunk, double *C, int64_t ldc, double alpha,
            double beta, double *part, int c0, int c1, const int *abort, hipStream_t s,
            unsigned long long *rec, int rec_off) {
  OzDesc d{};
  d.rec = rec;
  d.rec_off = rec_off;
  d.PA = PA; d.PB = PB; d.ea = ea; d.eb = eb;
  d.M = M; d.N = N; d.Kp = Kp; d.L0 = L0; d.kchunk = kchunk;
  d.C = C; d.ldc = ldc; d.alpha = alpha; d.beta = beta; d.part = part;
  d.c0 = c0; d.c1 = c1; d.abort = abort;
  // the SYR2K's planes and exponents are those of the rows from C's first
  // (the caller offsets C, op(A) and op(B) to the column range's start)
  if (epi == E_SYR2K && c0 != 0) return BANDRED_ERR_UNSUPPORTED;
  if (epi == E_SYR2K) {
    const int rows = M - c0, cols = c1 - c0;
    if (rows <= 0 || cols <= 0) return 0;
    d.nI = (rows + 63) / 64; d.nJ = (cols + 63) / 64; d.nZ = 1;
  } else {
    d.nI = (M + 63) / 64; d.nJ = (N + 63) / 64; d.nZ = ksplit;
  }
  // lower tiles of the SYR2K (cols <= rows: column J has nI - J of them)
  const int64_t total = (epi == E_SYR2K)
                            ? (int64_t)d.nJ * d.nI - (int64_t)d.nJ * (d.nJ - 1) / 2
                            : (int64_t)d.nI * d.nJ * d.nZ;
  if (total > ((int64_t)1 << 30)) return BANDRED_ERR_UNSUPPORTED;
  const dim3 grid((unsigned)total);
  if (epi == E_SYR2K)
    hipLaunchKernelGGL(k_gemm_oz<E_SYR2K>, grid, dim3(256), 0, s, d);
  else if (epi == E_PART)
    hipLaunchKernelGGL(k_gemm_oz<E_PART>, grid, dim3(256), 0, s, d);
  else
    hipLaunchKernelGGL(k_gemm_oz<E_AXPBY>, grid, dim3(256), 0, s, d);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace br
