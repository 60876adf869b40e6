// gemm.hip -- LDS-tiled MFMA contractions of the trailing update (gfx950).
//
// One kernel template covers every product of the reductions:
//   SYMM   P = A2 * V                (eq. updateA2symm; A2 symmetric, lower stored)
//   SYR2K  A2 -= W V^T + V W^T       (eq. updateA2syr2k; lower triangle only)
//   GEMM   the small products of eqs. updateA2gemm1/gemm2, the left update of
//          eq. updateA1 and the left/right GEMM pairs of eqs. updateCD/updateD.
//
// Workgroup = 4 waves of 64 lanes arranged 2 x 2 over a BM x BN output tile;
// each wave owns a (BM/2) x (BN/2) sub-tile made of 16 x 16 MFMA blocks.  The
// k dimension is staged through LDS in slices of kBK = 16 with double
// buffering: the next slice is fetched from global memory into registers while
// the current one feeds the matrix cores.
//
// Precision forms (the trailing-update products only):
//   P_F64    v_mfma_f64_16x16x4_f64, FP64 accumulation.
//   P_F32    operands rounded to FP32 while staged, v_mfma_f32_16x16x4_f32,
//            FP32 accumulation over the whole k range.
//   P_SPLIT  x = hi + lo with hi = fl32(x), lo = fl32(x - hi); three FP32 MFMA
//            products hi*hi, hi*lo, lo*hi (lo*lo dropped) into two FP32
//            accumulators that are folded into FP64 after every k slice:
//            acc64 += (double)(hi*lo + lo*hi) + (double)(hi*hi).
#include "common.hpp"

namespace br {

// MFMA 16x16x4 operand layout: lane l supplies A(l % 16, l / 16) and
// B(l / 16, l % 16); the result D(i, j) sits in lane j + 16 * f(i), element g(i):
//   v_mfma_f64_16x16x4_f64: lane l, element e holds row (l / 16) + 4 e
//   v_mfma_f32_16x16x4_f32: lane l, element e holds row 4 (l / 16) + e
// (both measured on gfx950), column l % 16 in both cases.
template <int PREC>
__device__ __forceinline__ int mfma_row(int lane, int e) {
  return (PREC == P_F64) ? (lane >> 4) + 4 * e : 4 * (lane >> 4) + e;
}
__device__ __forceinline__ int mfma_col(int lane) { return lane & 15; }

template <int PREC> struct Stage;
template <> struct Stage<P_F64> {
  using T = double;
  static constexpr int NPARTS = 1;
};
template <> struct Stage<P_F32> {
  using T = float;
  static constexpr int NPARTS = 1;
};
template <> struct Stage<P_SPLIT> {
  using T = float;
  static constexpr int NPARTS = 2;  // hi, lo
};

// ---------------------------------------------------------------------------
// operand fetch (global -> registers) with the coalescing-friendly mapping
// ---------------------------------------------------------------------------

// mapping 0: index fastest along the tile's M (or N) side; mapping 1: along k.
template <int BMN>
__device__ __forceinline__ void map_elem(int mapping, int idx, int &mn, int &kk) {
  if (mapping == 0) {
    mn = idx % BMN;
    kk = idx / BMN;
  } else {
    kk = idx % kBK;
    mn = idx / kBK;
  }
}

template <int BM, int OPA>
__device__ __forceinline__ int a_mapping(int i0, int k0) {
  if (OPA == A_N) return 0;
  if (OPA == A_T) return 1;
  // A_SYM: below the diagonal the stored element (i,k) is contiguous in i,
  // above it the element (k,i) is contiguous in k.
  if (k0 + kBK - 1 <= i0) return 0;
  if (k0 >= i0 + BM - 1) return 1;
  return 0;
}

template <int BM, int OPA>
__device__ __forceinline__ void fetch_a(const GemmDesc &d, int i0, int k0, int kend, int mapping,
                                        double *ra) {
  constexpr int E = BM * kBK / kThreads;
  const int tid = threadIdx.x;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    int ii, kk;
    map_elem<BM>(mapping, tid + kThreads * e, ii, kk);
    const int i = i0 + ii, k = k0 + kk;
    double v = 0.0;
    if (i < d.M && k < kend) {
      int64_t off;
      if (OPA == A_N) off = i + (int64_t)k * d.lda;
      else if (OPA == A_T) off = k + (int64_t)i * d.lda;
      else off = (i >= k) ? (i + (int64_t)k * d.lda) : (k + (int64_t)i * d.lda);
      v = d.A[off];
    }
    ra[e] = v;
  }
}

template <int BN, int OPB>
__device__ __forceinline__ int b_mapping() {
  return (OPB == B_N) ? 1 : 0;
}

template <int BN, int OPB>
__device__ __forceinline__ void fetch_b(const GemmDesc &d, int j0, int k0, int kend, double *rb) {
  constexpr int E = BN * kBK / kThreads;
  const int tid = threadIdx.x;
  const int mapping = b_mapping<BN, OPB>();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    int jj, kk;
    map_elem<BN>(mapping, tid + kThreads * e, jj, kk);
    const int j = j0 + jj, k = k0 + kk;
    double v = 0.0;
    if (j < d.N && k < kend) {
      int64_t off;
      if (OPB == B_N) off = k + (int64_t)j * d.ldb;
      else if (OPB == B_T) off = j + (int64_t)k * d.ldb;
      else {
        int kr = k + d.rot;
        if (kr >= d.K) kr -= d.K;
        off = j + (int64_t)kr * d.ldb;
      }
      v = d.B[off];
    }
    rb[e] = v;
  }
}

// Interior slices (the whole tile side in range, a full k slice, no diagonal
// crossing for the symmetric operand) take a fast path: one uniform base per
// slice plus a per-thread 32-bit element offset, without bounds tests, so the
// loads go out as a short run of global loads with a scalar base.
typedef __attribute__((address_space(1))) double gdbl;
typedef __attribute__((address_space(1))) char gchr;
__device__ __forceinline__ double gload(const double *p, uint32_t i) {
  return *(const gdbl *)((const gchr *)p + (i << 3));
}

// A_SYM slice wholly below (mapping 0) or wholly above (mapping 1) the
// diagonal; the plain operands are always pure
template <int BM, int OPA>
__device__ __forceinline__ bool a_pure(int i0, int k0) {
  if (OPA != A_SYM) return true;
  return (k0 + kBK - 1 <= i0) || (k0 >= i0 + BM - 1);
}

template <int BM, int OPA>
__device__ __forceinline__ void fetch_a_fast(const GemmDesc &d, int i0, int k0, int mapping,
                                             double *ra) {
  constexpr int E = BM * kBK / kThreads;
  const int tid = threadIdx.x;
  // element (i, k) of op(A): stored at (i, k) for A_N and the lower part of
  // A_SYM, at (k, i) for A_T and the upper part
  const bool stored_ik = (OPA == A_N) || (OPA == A_SYM && mapping == 0);
  const double *base = stored_ik ? d.A + i0 + (int64_t)k0 * d.lda : d.A + k0 + (int64_t)i0 * d.lda;
  const uint32_t ld = (uint32_t)d.lda;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    int ii, kk;
    map_elem<BM>(mapping, tid + kThreads * e, ii, kk);
    const uint32_t off = stored_ik ? (uint32_t)ii + (uint32_t)kk * ld : (uint32_t)kk + (uint32_t)ii * ld;
    ra[e] = gload(base, off);
  }
}

template <int BN, int OPB>
__device__ __forceinline__ void fetch_b_fast(const GemmDesc &d, int j0, int k0, double *rb) {
  constexpr int E = BN * kBK / kThreads;
  const int tid = threadIdx.x;
  const int mapping = b_mapping<BN, OPB>();
  int kb = k0;
  if (OPB == B_TROT) {  // rot and K multiples of kBK: no wrap inside the slice
    kb = k0 + d.rot;
    if (kb >= d.K) kb -= d.K;
  }
  const double *base = (OPB == B_N) ? d.B + k0 + (int64_t)j0 * d.ldb : d.B + j0 + (int64_t)kb * d.ldb;
  const uint32_t ld = (uint32_t)d.ldb;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    int jj, kk;
    map_elem<BN>(mapping, tid + kThreads * e, jj, kk);
    const uint32_t off = (OPB == B_N) ? (uint32_t)kk + (uint32_t)jj * ld : (uint32_t)jj + (uint32_t)kk * ld;
    rb[e] = gload(base, off);
  }
}

// registers -> LDS, converting to the stage type (hi/lo split for P_SPLIT)
template <int BMN, int PREC, int LD>
__device__ __forceinline__ void stash(typename Stage<PREC>::T *lds, int part_stride, int mapping,
                                      const double *r) {
  constexpr int E = BMN * kBK / kThreads;
  const int tid = threadIdx.x;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    int mn, kk;
    map_elem<BMN>(mapping, tid + kThreads * e, mn, kk);
    const int o = kk * LD + mn;
    if (PREC == P_F64) {
      lds[o] = r[e];
    } else if (PREC == P_F32) {
      lds[o] = (float)r[e];
    } else {
      const float hi = (float)r[e];
      const float lo = (float)(r[e] - (double)hi);
      lds[o] = hi;
      lds[o + part_stride] = lo;
    }
  }
}

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------

template <int BM, int BN, int OPA, int OPB, int EPI, int PREC>
__global__ __launch_bounds__(kThreads, 2) void k_gemm(GemmDesc d) {
  using T = typename Stage<PREC>::T;
  constexpr int NP = Stage<PREC>::NPARTS;
  constexpr int LDA_S = BM + 1;  // odd stride: transposed stores spread over banks
  constexpr int LDB_S = BN + 1;
  constexpr int SA = kBK * LDA_S;  // one part of one A stage
  constexpr int SB = kBK * LDB_S;
  constexpr int FM = BM / 32, FN = BN / 32;  // 16x16 blocks per wave
  constexpr int EA = BM * kBK / kThreads, EB = BN * kBK / kThreads;

  __shared__ T As[2 * NP * SA];
  __shared__ T Bs[2 * NP * SB];

  if (d.gate && *d.gate != d.gate_val) return;
  if (d.abort && *d.abort != 0) return;
  if (d.prio) __builtin_amdgcn_s_setprio(kPrioPanel);
  int i0, j0, kbeg, kend;
  if (EPI == E_SYR2K) {
    const int I = blockIdx.x, J = blockIdx.y;
    if ((I + 1) * BM - 1 < J * BN) return;  // tile entirely above the diagonal
    i0 = d.c0 + I * BM;
    j0 = d.c0 + J * BN;
    kbeg = 0;
    kend = d.K;
  } else {
    i0 = blockIdx.x * BM;
    j0 = blockIdx.y * BN;
    kbeg = blockIdx.z * d.kchunk;
    kend = min(d.K, kbeg + d.kchunk);
  }
  const int Nlim = (EPI == E_SYR2K) ? d.c1 : d.N;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  // accumulators
  v4d acc64[FM][FN];
  v4f acc32[FM][FN];
  v4f accx[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      acc64[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
      acc32[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
      accx[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    }

  double ra[EA], rb[EB];
  GemmDesc dd = d;
  if (EPI == E_SYR2K) dd.N = d.c1;  // B operand rows are indexed by C's column

  const int nst = (kend - kbeg + kBK - 1) / kBK;
  // fast loads: whole tile sides in range and 32-bit offsets within a slice
  const int64_t ldmax = d.lda > d.ldb ? d.lda : d.ldb;
  const bool rot_ok = (OPB != B_TROT) || ((d.rot | d.K) & (kBK - 1)) == 0;
  const bool fast_tile = (i0 + BM <= dd.M) && (j0 + BN <= dd.N) && rot_ok &&
                         ldmax * (BM > BN ? BM : BN) < ((int64_t)1 << 28);
  auto fetch = [&](int k0, int mapping) {
    if (fast_tile && k0 + kBK <= kend && a_pure<BM, OPA>(i0, k0)) {
      fetch_a_fast<BM, OPA>(dd, i0, k0, mapping, ra);
      fetch_b_fast<BN, OPB>(dd, j0, k0, rb);
    } else {
      fetch_a<BM, OPA>(dd, i0, k0, kend, mapping, ra);
      fetch_b<BN, OPB>(dd, j0, k0, kend, rb);
    }
  };
  if (nst > 0) {
    int mapA = a_mapping<BM, OPA>(i0, kbeg);
    fetch(kbeg, mapA);
    stash<BM, PREC, LDA_S>(As, SA, mapA, ra);
    stash<BN, PREC, LDB_S>(Bs, SB, b_mapping<BN, OPB>(), rb);
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
      const int buf = s & 1;
      const bool more = (s + 1 < nst);
      int mapN = 0;
      if (more) {
        const int k0 = kbeg + (s + 1) * kBK;
        mapN = a_mapping<BM, OPA>(i0, k0);
        fetch(k0, mapN);
      }
      const T *as = As + buf * NP * SA;
      const T *bs = Bs + buf * NP * SB;
#pragma unroll
      for (int kq = 0; kq < kBK; kq += 4) {
        const int ka = (kq + (lane >> 4));
        T a[FM], b[FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm) a[fm] = as[ka * LDA_S + wm * (BM / 2) + fm * 16 + (lane & 15)];
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) b[fn] = bs[ka * LDB_S + wn * (BN / 2) + fn * 16 + (lane & 15)];
        if constexpr (PREC == P_F64) {
#pragma unroll
          for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn)
              acc64[fm][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[fn], a[fm], acc64[fm][fn], 0, 0, 0);
        } else if constexpr (PREC == P_F32) {
#pragma unroll
          for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn)
              acc32[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[fn], a[fm], acc32[fm][fn], 0, 0, 0);
        } else {
          float al[FM], bl[FN];
#pragma unroll
          for (int fm = 0; fm < FM; ++fm) al[fm] = as[SA + ka * LDA_S + wm * (BM / 2) + fm * 16 + (lane & 15)];
#pragma unroll
          for (int fn = 0; fn < FN; ++fn) bl[fn] = bs[SB + ka * LDB_S + wn * (BN / 2) + fn * 16 + (lane & 15)];
#pragma unroll
          for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
              acc32[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[fn], a[fm], acc32[fm][fn], 0, 0, 0);
              accx[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x4f32(bl[fn], a[fm], accx[fm][fn], 0, 0, 0);
              accx[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[fn], al[fm], accx[fm][fn], 0, 0, 0);
            }
        }
      }
      if constexpr (PREC == P_SPLIT) {
        // fold this slice's FP32 partial sums into the FP64 accumulator
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
          for (int fn = 0; fn < FN; ++fn) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              acc64[fm][fn][e] += (double)accx[fm][fn][e] + (double)acc32[fm][fn][e];
            acc32[fm][fn] = v4f{0.f, 0.f, 0.f, 0.f};
            accx[fm][fn] = v4f{0.f, 0.f, 0.f, 0.f};
          }
      }
      if (more) {
        T *asn = As + (buf ^ 1) * NP * SA;
        T *bsn = Bs + (buf ^ 1) * NP * SB;
        stash<BM, PREC, LDA_S>(asn, SA, mapN, ra);
        stash<BN, PREC, LDB_S>(bsn, SB, b_mapping<BN, OPB>(), rb);
      }
      __syncthreads();
    }
  }
  if constexpr (PREC == P_F32) {
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc64[fm][fn][e] = (double)acc32[fm][fn][e];
  }

  // epilogue.  C is read in groups of 16 values (one fm row of blocks), two
  // groups in flight: the loads of group fm + 1 go out before group fm is
  // stored (the registers of the operand staging are free by now), so the
  // read latency is paid about once per tile instead of once per group.
  const bool readC = (EPI == E_SYR2K) || (EPI == E_AXPBY && d.beta != 0.0);
  // the MFMA computed the transposed block (B^T A^T): its row index is C's
  // column, its column index (lane % 16) is C's row, so 16 adjacent lanes
  // touch 16 adjacent rows of one column (128 contiguous bytes)
  auto row_of = [&](int fm) { return i0 + wm * (BM / 2) + fm * 16 + mfma_col(lane); };
  auto col_of = [&](int fn, int e) { return j0 + wn * (BN / 2) + fn * 16 + mfma_row<PREC>(lane, e); };
  auto inside = [&](int row, int col) {
    bool in = (row < d.M && col < Nlim);
    if (EPI == E_SYR2K) in = in && (row >= col);
    return in;
  };
  double cv[2][FN][4];
  auto load_c = [&](int fm, double (&c)[FN][4]) {
    const int row = row_of(fm);
#pragma unroll
    for (int fn = 0; fn < FN; ++fn)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int col = col_of(fn, e);
        const bool in = inside(row, col);
        const double x = d.C[in ? row + (int64_t)col * d.ldc : 0];  // clamped, no branch
        c[fn][e] = in ? x : 0.0;
      }
  };
  if (readC) load_c(0, cv[0]);
#pragma unroll
  for (int fm = 0; fm < FM; ++fm) {
    if (readC && fm + 1 < FM) load_c(fm + 1, cv[(fm + 1) & 1]);
    const int row = row_of(fm);
#pragma unroll
    for (int fn = 0; fn < FN; ++fn)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int col = col_of(fn, e);
        if (!inside(row, col)) continue;
        const double v = acc64[fm][fn][e];
        const double c = cv[fm & 1][fn][e];
        if (EPI == E_AXPBY) {
          const double o = readC ? d.alpha * v + d.beta * c : d.alpha * v;
          d.C[row + (int64_t)col * d.ldc] = o;
          if (d.C2) {
            if (d.c2_trans) d.C2[col + (int64_t)row * d.ldc2] = o;
            else d.C2[row + (int64_t)col * d.ldc2] = o;
          }
        } else if (EPI == E_PART) {
          d.part[(int64_t)blockIdx.z * d.M * d.N + row + (int64_t)col * d.M] = v;
        } else {
          d.C[row + (int64_t)col * d.ldc] = c - v;
        }
      }
  }
}

__global__ void k_reduce_partials(const double *part, int ksplit, int M, int N, double alpha,
                                  double *C, int64_t ldc, double beta, const int *gate,
                                  int gate_val, const int *abort) {
  if (gate && *gate != gate_val) return;
  if (abort && *abort != 0) return;
  __builtin_amdgcn_s_setprio(kPrioPanel);  // split-k sums: on the panel chain or alone
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    // the partials are loaded eight at a time (independent loads, one memory
    // latency per group instead of per partial) and summed in z order
    double s = 0.0;
    int z = 0;
    for (; z + 8 <= ksplit; z += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(z + u) * total + idx];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; z < ksplit; ++z) s += part[z * total + idx];
    const int64_t i = idx % M, j = idx / M;
    double *c = C + i + j * ldc;
    *c = (beta == 0.0) ? alpha * s : alpha * s + beta * (*c);
  }
}

__global__ void k_fill(double *p, int64_t count, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u32(unsigned *p, int64_t count, unsigned v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

template <int BM, int BN, int OPA, int OPB, int EPI, int PREC>
static int launch_t(const GemmDesc &d, int ksplit, hipStream_t s) {
  dim3 grid;
  if (EPI == E_SYR2K) {
    const int rows = d.M - d.c0, cols = d.c1 - d.c0;
    if (rows <= 0 || cols <= 0) return 0;
    grid = dim3((rows + BM - 1) / BM, (cols + BN - 1) / BN, 1);
  } else {
    if (d.M <= 0 || d.N <= 0) return 0;
    grid = dim3((d.M + BM - 1) / BM, (d.N + BN - 1) / BN, ksplit);
  }
  hipLaunchKernelGGL((k_gemm<BM, BN, OPA, OPB, EPI, PREC>), grid, dim3(kThreads), d.lds_pad, s, d);
  return 0;
}

template <int BM, int BN, int PREC>
static int dispatch_ops(int opa, int opb, int epi, const GemmDesc &d, int ksplit, hipStream_t s) {
#define BR_CASE(OA, OB, EP) \
  if (opa == OA && opb == OB && epi == EP) return launch_t<BM, BN, OA, OB, EP, PREC>(d, ksplit, s);
  BR_CASE(A_SYM, B_N, E_PART)
  BR_CASE(A_SYM, B_N, E_AXPBY)
  BR_CASE(A_N, B_N, E_AXPBY)
  BR_CASE(A_N, B_N, E_PART)
  BR_CASE(A_T, B_N, E_AXPBY)
  BR_CASE(A_T, B_N, E_PART)
  BR_CASE(A_N, B_T, E_AXPBY)
  BR_CASE(A_N, B_T, E_PART)
  BR_CASE(A_N, B_TROT, E_SYR2K)
#undef BR_CASE
  return BANDRED_ERR_UNSUPPORTED;
}

// Rectangular tiles for products with one narrow output side (no SYR2K).
template <int BM, int BN, int PREC>
static int dispatch_rect(int opa, int opb, int epi, const GemmDesc &d, int ksplit, hipStream_t s) {
#define BR_CASE(OA, OB, EP) \
  if (opa == OA && opb == OB && epi == EP) return launch_t<BM, BN, OA, OB, EP, PREC>(d, ksplit, s);
  BR_CASE(A_SYM, B_N, E_PART)
  BR_CASE(A_SYM, B_N, E_AXPBY)
  BR_CASE(A_N, B_N, E_AXPBY)
  BR_CASE(A_N, B_N, E_PART)
  BR_CASE(A_T, B_N, E_AXPBY)
  BR_CASE(A_T, B_N, E_PART)
  BR_CASE(A_N, B_T, E_AXPBY)
  BR_CASE(A_N, B_T, E_PART)
#undef BR_CASE
  return BANDRED_ERR_UNSUPPORTED;
}

int gemm_tile_shape(int epi, int M, int N, int tile64, int *tm, int *tn) {
  // 64 x 64 tiles for outputs up to 128 x 128 (the b x b products and Gram
  // matrices), so that such products still spread over several workgroups,
  // and when the caller asks for them (products with fewer 128 x 128 tiles
  // than CUs and no k split); 128 x 64 (64 x 128) when the output has at most
  // 64 columns (rows), so that no wave computes a block of zero columns
  if (tile64 || (M <= 128 && N <= 128)) {
    *tm = 64; *tn = 64;
  } else if (epi != E_SYR2K && N <= 64) {
    *tm = 128; *tn = 64;
  } else if (epi != E_SYR2K && M <= 64) {
    *tm = 64; *tn = 128;
  } else {
    *tm = 128; *tn = 128;
  }
  return 0;
}

int launch_gemm(int opa, int opb, int epi, int prec, const GemmDesc &d, int ksplit,
                hipStream_t s) {
  int tm = 128, tn = 128;
  gemm_tile_shape(epi, d.M, epi == E_SYR2K ? (d.c1 - d.c0) : d.N, d.tile64, &tm, &tn);
  int rc;
  if (prec == P_F64) {
    rc = (tm == 64 && tn == 64) ? dispatch_ops<64, 64, P_F64>(opa, opb, epi, d, ksplit, s)
         : (tn == 64)           ? dispatch_rect<128, 64, P_F64>(opa, opb, epi, d, ksplit, s)
         : (tm == 64)           ? dispatch_rect<64, 128, P_F64>(opa, opb, epi, d, ksplit, s)
                                : dispatch_ops<128, 128, P_F64>(opa, opb, epi, d, ksplit, s);
  } else if (prec == P_F32) {
    rc = (tm == 64 && tn == 64) ? dispatch_ops<64, 64, P_F32>(opa, opb, epi, d, ksplit, s)
         : (tn == 64)           ? dispatch_rect<128, 64, P_F32>(opa, opb, epi, d, ksplit, s)
         : (tm == 64)           ? dispatch_rect<64, 128, P_F32>(opa, opb, epi, d, ksplit, s)
                                : dispatch_ops<128, 128, P_F32>(opa, opb, epi, d, ksplit, s);
  } else {
    rc = dispatch_ops<64, 64, P_SPLIT>(opa, opb, epi, d, ksplit, s);
  }
  if (rc != 0) return rc;
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

int launch_reduce_partials(const double *part, int ksplit, int M, int N, double alpha,
                           double *C, int64_t ldc, double beta, hipStream_t s, const int *gate,
                           int gate_val, const int *abort) {
  const int64_t total = (int64_t)M * N;
  if (total <= 0) return 0;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_reduce_partials, dim3(blocks), dim3(256), 0, s, part, ksplit, M, N, alpha,
                     C, ldc, beta, gate, gate_val, abort);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

int launch_fill(double *p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return 0;
  int blocks = (int)((count + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, p, count, v);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

int launch_fill_u32(unsigned *p, int64_t count, unsigned v, hipStream_t s) {
  if (count <= 0) return 0;
  int blocks = (int)((count + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, count, v);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace br
