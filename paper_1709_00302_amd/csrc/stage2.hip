// stage2.hip -- the steps after the band reduction in a two-stage symmetric
// eigenvalue solver (gfx950): band -> tridiagonal by Householder bulge
// chasing, and the eigenvalues of the tridiagonal matrix by multisection on
// Sturm counts.  The paper times this pipeline with SBR's band-to-tridiagonal
// routine and LAPACK's DSTERF after its first stage (Sec. 4.3).
//
// Band to tridiagonal.  The symmetric band B (bandwidth w) is copied into a
// band store with room for the bulges: AB(k, c) = B(c + k, c), 0 <= k <= 2w.
// Sweep s makes column s tridiagonal: step 0 builds the reflector that
// annihilates B(s+2 : s+w, s) (rows S0 = s+1 .. s+w) and applies it to the
// diagonal block S0 x S0 from both sides and to the block R1 x S0 below it
// (R1 = s+w+1 .. s+2w) from the right, which fills R1 x S0 (the bulge).  Step
// k >= 1 annihilates the first column of that bulge below its first row
// (rows R_k = s+1+kw .. s+(k+1)w, column s+1+(k-1)w) with a reflector on R_k,
// applies it from the left to the rest of the bulge block, from both sides to
// R_k x R_k and from the right to the next block R_{k+1} x R_k, pushing the
// bulge w rows down.  The rest of each bulge block is annihilated by the
// following sweeps (their blocks are shifted by one row and column), so the
// matrix never has more than 2w subdiagonals.
//
// Sweeps run concurrently: one persistent workgroup per sweep at a time,
// sweeps claimed in increasing order from an atomic counter.  Step k >= 1 of
// sweep s touches the elements (r, c) with r in s+1+kw .. s+(k+2)w and c in
// s+1+(k-1)w .. s+(k+1)w (step 0: rows s+1 .. s+2w, columns s .. s+w): its
// rows s+1+kw .. s+(k+1)w (the reflector's column, the bulge block and the
// diagonal block) meet only steps k-1 .. k+1 of sweep s-1, its block below
// (rows s+1+(k+1)w ..) steps k .. k+2.  A step publishes itself once its rows
// s+1+kw .. s+(k+1)w are stored, before it updates its block below (whose
// stores the next step's publication covers; a sweep's last step has no
// block below).  So step k begins once sweep s-1 has published k+2 steps and
// loads its block below once it has published k+3; meanwhile sweep s-1's
// later work stays below row s+(k+2)w, clear of everything step k touches
// until then, so every element sees the operations of the sequential order,
// in that order.  The waits are bounded (wall clock), and a workgroup that
// gives up raises an abort flag that releases every other one.
#include "common.hpp"

namespace br {

constexpr int kS2T = 512;      // threads of the bulge-chasing workgroup (8 waves)
constexpr int kS2LD = kNbMax + 1;  // row stride of the LDS block (odd: no bank conflicts)

struct Sb2stDesc {
  double *AB;
  int64_t ldab;
  int n, w, nsweeps;
  unsigned *sweep_ctr;
  int *progress;               // steps finished per sweep
  int *status, *abort_flag;
  long long timeout_ticks;
};

__device__ __forceinline__ int sweep_steps(int n, int w, int s) {
  // steps k = 0 .. K-1 with s + 1 + k w < n for k >= 1
  const int rem = n - 1 - s;  // > 0
  return 1 + (rem > w ? (rem - 1) / w : 0);
}

constexpr int kS2G = kS2T / kNbMax;  // thread groups sharing one matrix-vector product

struct S2Lds {
  double blk[kNbMax * kS2LD];  // one block of the step, row-major blk[r * kS2LD + c]
  double v[kNbMax];
  double p[kNbMax];
  double part[kS2G][kNbMax];   // partial sums of the matrix-vector products
  double red[kS2T / 64];
  int go;
  int sweep;
};

// out[x] = scale * sum_y M(x, y) v[y] for x < nx, y < ny, with M(x, y) =
// blk[x * kS2LD + y] (rows, trans = 0) or blk[y * kS2LD + x] (columns,
// trans = 1): kS2G groups of kNbMax threads each take a quarter of y, then
// the partial sums are added.  Ends with a barrier.
__device__ __forceinline__ void blk_matvec(S2Lds &sh, int trans, int nx, int ny, double scale,
                                           double *out) {
  const int g = threadIdx.x / kNbMax, x = threadIdx.x % kNbMax;
  const int per = (ny + kS2G - 1) / kS2G, y0 = g * per, y1 = min(ny, y0 + per);
  if (x < nx) {
    double acc = 0.0;
    for (int y = y0; y < y1; ++y)
      acc += (trans ? sh.blk[y * kS2LD + x] : sh.blk[x * kS2LD + y]) * sh.v[y];
    sh.part[g][x] = acc;
  }
  __syncthreads();
  if (threadIdx.x < nx) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kS2G; ++i) t += sh.part[i][threadIdx.x];
    out[threadIdx.x] = scale * t;
  }
  __syncthreads();
}

__device__ __forceinline__ double block_sum(double x, double *red) {
  // all threads of the workgroup; result in every thread
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wv] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kS2T / 64; ++i) t += red[i];
  return t;
}

// The elements (t, j), t < rows, j < cols, of a block in column-major order,
// kS2T apart: thread tid's q-th element is tid + q kS2T.  The (t, j) pairs
// are stepped without integer division.
struct Walk {
  int t, j, dt, dj, rows;
  __device__ Walk(int rows_) : rows(rows_) {
    t = threadIdx.x % rows_;
    j = threadIdx.x / rows_;
    dt = kS2T % rows_;
    dj = kS2T / rows_;
  }
  __device__ __forceinline__ void next() {
    t += dt;
    j += dj;
    if (t >= rows) {
      t -= rows;
      ++j;
    }
  }
};

// Band-store accesses of the bulge chasing: relaxed atomics at agent scope.
// The sweeps hand their blocks to one another across workgroups (possibly on
// different XCDs, whose L2 caches are not coherent with each other); with
// these accesses the data does not sit dirty in one XCD's L2, so the release
// and acquire fences of the progress hand-off stay cheap.
__device__ __forceinline__ double bld(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void bst(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A rows x cols block of the band store whose element (t, j) is the matrix
// element (r0 + t, c0 + j), at AB + (r0 + t) + (c0 + j)(ld - 1).  When rows
// divides the workgroup (every full block for w = 32, 64, 128) a thread keeps
// row t = tid % rows and takes the columns j = tid / rows + q dj, dj = kS2T /
// rows: its addresses step by the uniform stride dj (ld - 1) and its row's
// entries of v and p stay in registers.  Other shapes (the shorter blocks at
// the end of a sweep) walk the elements in column-major order, kS2T apart.
struct BandBlk {
  double *AB;
  int64_t ld;
  int r0, c0, rows, cols;
  __device__ __forceinline__ double *at(int t, int j) const {
    return AB + (int64_t)(r0 + t) + (int64_t)(c0 + j) * (ld - 1);
  }
};
constexpr int kS2Per = (kNbMax * kNbMax + kS2T - 1) / kS2T;  // elements per thread

// The loads of a block in two halves, so that other work can run while they
// are in flight: blk_fetch issues the loads of the elements with keep(t, j)
// into r[], blk_place hands the arrived values to dst(t, j, value).
template <class Keep>
__device__ __forceinline__ void blk_fetch(const BandBlk &b, Keep keep, double (&r)[kS2Per]) {
  if (kS2T % b.rows == 0) {
    const int t = threadIdx.x % b.rows, j0 = threadIdx.x / b.rows, dj = kS2T / b.rows;
    const double *p = b.at(t, j0);
    const int64_t step = (int64_t)dj * (b.ld - 1);
#pragma unroll
    for (int q = 0; q < kS2Per; ++q) {
      const int j = j0 + q * dj;
      r[q] = (j < b.cols && keep(t, j)) ? bld(p + q * step) : 0.0;
    }
    return;
  }
  Walk a(b.rows);
#pragma unroll
  for (int q = 0; q < kS2Per; ++q) {
    r[q] = (a.j < b.cols && keep(a.t, a.j)) ? bld(b.at(a.t, a.j)) : 0.0;
    a.next();
  }
}
template <class Keep, class Dst>
__device__ __forceinline__ void blk_place(const BandBlk &b, Keep keep, const double (&r)[kS2Per],
                                          Dst dst) {
  if (kS2T % b.rows == 0) {
    const int t = threadIdx.x % b.rows, j0 = threadIdx.x / b.rows, dj = kS2T / b.rows;
#pragma unroll
    for (int q = 0; q < kS2Per; ++q) {
      const int j = j0 + q * dj;
      if (j < b.cols && keep(t, j)) dst(t, j, r[q]);
    }
    return;
  }
  Walk c(b.rows);
#pragma unroll
  for (int q = 0; q < kS2Per; ++q) {
    if (c.j < b.cols && keep(c.t, c.j)) dst(c.t, c.j, r[q]);
    c.next();
  }
}
template <class Keep, class Dst>
__device__ __forceinline__ void blk_load(const BandBlk &b, Keep keep, Dst dst) {
  double r[kS2Per];
  blk_fetch(b, keep, r);
  blk_place(b, keep, r, dst);
}

// value(t, j) to the elements with keep(t, j), and with WB also to
// blk[t][j].  value() only reads LDS; on the fast path a thread forms half of
// its values (their LDS reads in flight together) before it stores them.
template <bool WB, class Keep, class Val>
__device__ __forceinline__ void blk_store(const BandBlk &b, double *blk, Keep keep, Val value) {
  if (kS2T % b.rows == 0) {
    const int t = threadIdx.x % b.rows, j0 = threadIdx.x / b.rows, dj = kS2T / b.rows;
    double *p = b.at(t, j0);
    const int64_t step = (int64_t)dj * (b.ld - 1);
    constexpr int H = kS2Per / 2;
#pragma unroll
    for (int h = 0; h < kS2Per; h += H) {
      double x[H];
#pragma unroll
      for (int q = 0; q < H; ++q) x[q] = value(t, min(j0 + (h + q) * dj, b.cols - 1));
#pragma unroll
      for (int q = 0; q < H; ++q) {
        const int j = j0 + (h + q) * dj;
        if (j < b.cols && keep(t, j)) {
          if (WB) blk[t * kS2LD + j] = x[q];
          bst(p + (h + q) * step, x[q]);
        }
      }
    }
    return;
  }
  Walk a(b.rows);
  for (int q = 0; q < kS2Per && a.j < b.cols; ++q) {
    if (keep(a.t, a.j)) {
      const double x = value(a.t, a.j);
      if (WB) blk[a.t * kS2LD + a.j] = x;
      bst(b.at(a.t, a.j), x);
    }
    a.next();
  }
}

__device__ __forceinline__ long long s2_ticks() { return (long long)wall_clock64(); }

// Wait, with the whole workgroup, until sweep s-1 has finished `need` steps:
// thread 0 polls the progress word relaxed and acquires once at agent scope,
// and the barrier orders the other threads after it.  False when the wait
// gave up (its time limit, or another workgroup's abort).
__device__ __forceinline__ bool wait_prev(const Sb2stDesc &d, S2Lds &sh, int s, int need) {
  if (threadIdx.x == 0) {
    int ok = 1;
    const long long t0 = s2_ticks();
    while (__hip_atomic_load(d.progress + (s - 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
           need) {
      if (__hip_atomic_load(d.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      if (s2_ticks() - t0 > d.timeout_ticks) {
        __hip_atomic_store(d.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(d.status, (int)BANDRED_ERR_TIMEOUT, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    sh.go = ok;
  }
  __syncthreads();
  return sh.go != 0;
}

// one step (s, k) of the bulge chasing.  Every block the step touches is
// brought into LDS with coalesced loads (a column of a block is a contiguous
// piece of a band-store column), updated there and written back.
// kept: blk holds the block below of step k - 1 of this sweep as it was
// written back (rows rx .., columns cx ..): this step's column and bulge
// block, which no other sweep changes in between (the earlier sweep's work on
// it was published before step k - 1 loaded it, and the next sweep touches it
// only after this step has published)
// need_below: progress of sweep s-1 required before the block below is
// loaded (0: none).
// The step publishes itself (progress of sweep s = k + 1) as soon as its rows
// rx .. rx+L-1 are stored, before it updates the block below: a step of the
// next sweep waits only on such rows and on the blocks below of earlier steps,
// whose stores the same release covers (and a sweep's last step has no block
// below).  Returns kS2Kept when the step left its own block below in blk, and
// kS2Published once it has published; 0 when it ended early (a trivial
// reflector, or a wait that gave up, which leaves sh.go = 0).
constexpr int kS2Kept = 1, kS2Published = 2;
__device__ __forceinline__ int sb2st_step(const Sb2stDesc &d, S2Lds &sh, int s, int k,
                                          bool kept, int need_below) {
  const int n = d.n, w = d.w, tid = threadIdx.x;
  const int64_t ld = d.ldab;
  double *AB = d.AB;
  auto ptr = [&](int r, int c) { return AB + ((int64_t)(r - c) + (int64_t)c * ld); };
  auto get = [&](int r, int c) { return bld(ptr(r, c)); };
  auto put = [&](int r, int c, double v) { bst(ptr(r, c), v); };
  auto all = [](int, int) { return true; };
  auto lower = [](int t, int u) { return t >= u; };
  int cx, rx, L;
  if (k == 0) {
    cx = s;
    rx = s + 1;
    L = min(w, n - 1 - s);
  } else {
    cx = s + 1 + (k - 1) * w;
    rx = s + 1 + k * w;
    L = min(w, n - rx);
  }
  if (L < 2) return 0;
  double *blk = sh.blk;
  // (1) the reflector that annihilates column cx below row rx
  double x = 0.0;
  if (tid < L) {
    x = kept ? blk[tid * kS2LD] : get(rx + tid, cx);
    sh.v[tid] = x;
  }
  const double sig2 = block_sum(tid >= 1 && tid < L ? x * x : 0.0, sh.red);
  const double alpha = sh.v[0];
  if (sig2 == 0.0) return 0;  // H = I
  const double nrm = sqrt(alpha * alpha + sig2);
  const double beta = (alpha < 0.0) ? nrm : -nrm;
  const double tau = (beta - alpha) / beta;
  const double dv = alpha - beta;
  __syncthreads();
  if (tid < L) {
    sh.v[tid] = (tid == 0) ? 1.0 : x / dv;
    put(rx + tid, cx, (tid == 0) ? beta : 0.0);
  }
  __syncthreads();
  // The diagonal block (rows and columns rx .. rx+L-1) and the block below
  // (rows rx+w .., columns rx .. rx+L-1) are final from the start of the
  // step: the steps of the previous sweep that write them have finished,
  // later sweeps wait for this one, and the stores this step makes before
  // loading them go to other rows or columns.  So their loads are issued
  // early, each hidden behind the phase before it.
  const BandBlk bd{AB, ld, rx, rx, L, L};
  const int r2 = rx + w;
  const int m2 = min(rx + 2 * w, n) - r2;
  const BandBlk bb{AB, ld, r2, rx, m2, L};
  double rd[kS2Per], rb[kS2Per];
  // (2) the rest of the bulge block, rows rx .. rx+L-1, columns cx+1 ..
  //     cx+w-1, from the left: B(rx + t, cx + 1 + j) = blk[t][j + o] with
  //     o = 1 for the kept block (its column 0 is column cx), else 0
  if (k >= 1) {
    const int nc = w - 1, o = kept ? 1 : 0;
    if (!kept) {
      blk_load(BandBlk{AB, ld, rx, cx + 1, L, nc}, all,
               [&](int t, int j, double a) { blk[t * kS2LD + j] = a; });
      __syncthreads();
    }
    blk_fetch(bd, lower, rd);
    // z_j = tau v^T blk(:, j): the columns o .. o + nc - 1 of blk
    {
      const int g = tid / kNbMax, xj = tid % kNbMax;
      const int per = (L + kS2G - 1) / kS2G, t0 = g * per, t1 = min(L, t0 + per);
      if (xj < nc) {
        double z = 0.0;
        for (int t = t0; t < t1; ++t) z += sh.v[t] * blk[t * kS2LD + xj + o];
        sh.part[g][xj] = z;
      }
      __syncthreads();
      if (tid < nc) {
        double z = 0.0;
#pragma unroll
        for (int i = 0; i < kS2G; ++i) z += sh.part[i][tid];
        sh.p[tid] = tau * z;
      }
      __syncthreads();
    }
    blk_store<false>(BandBlk{AB, ld, rx, cx + 1, L, nc}, blk, all, [&](int t, int j) {
      return blk[t * kS2LD + j + o] - sh.p[j] * sh.v[t];
    });
    __syncthreads();
  } else {
    blk_fetch(bd, lower, rd);
  }
  // (3) the diagonal block R x R from both sides: p = tau D v,
  //     q = p - (tau p^T v / 2) v, D -= v q^T + q v^T (lower part stored;
  //     the block is mirrored in LDS)
  blk_place(bd, lower, rd, [&](int t, int u, double a) {
    blk[t * kS2LD + u] = a;
    blk[u * kS2LD + t] = a;
  });
  if (m2 > 0 && need_below > 0) {
    if (!wait_prev(d, sh, s, need_below)) return 0;  // its barrier ends the placement
  } else {
    __syncthreads();
  }
  if (m2 > 0) blk_fetch(bb, all, rb);
  blk_matvec(sh, 0, L, L, tau, sh.p);  // p = tau D v
  const double pt = tid < L ? sh.p[tid] : 0.0;
  const double pv = block_sum(tid < L ? pt * sh.v[tid] : 0.0, sh.red);
  const double Kc = 0.5 * tau * pv;
  if (tid < L) sh.p[tid] = pt - Kc * sh.v[tid];  // q
  __syncthreads();
  blk_store<false>(bd, blk, lower, [&](int t, int u) {
    return blk[t * kS2LD + u] - (sh.v[t] * sh.p[u] + sh.p[t] * sh.v[u]);
  });
  // rows rx .. rx+L-1 are done: every thread's stores, then the progress word
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (tid == 0)
    __hip_atomic_store(d.progress + s, k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  // (4) the block below, rows rx+w .. rx+2w-1, from the right:
  //     blk[i][u] = B(r2 + i, rx + u)
  if (m2 > 0) {
    blk_place(bb, all, rb, [&](int i, int u, double a) { blk[i * kS2LD + u] = a; });
    __syncthreads();
    blk_matvec(sh, 0, m2, L, tau, sh.p);  // y = tau B v
    // updated in place and written back; the block stays in LDS for the
    // next step of this sweep
    blk_store<true>(bb, blk, all,
                    [&](int i, int u) { return blk[i * kS2LD + u] - sh.p[i] * sh.v[u]; });
    return kS2Kept | kS2Published;
  }
  return kS2Published;
}

__global__ __launch_bounds__(kS2T) void k_sb2st(Sb2stDesc d) {
  __shared__ S2Lds sh;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) {
      sh.sweep = (int)atomicAdd(d.sweep_ctr, 1u);
      sh.go = 1;
    }
    __syncthreads();
    const int s = sh.sweep;
    __syncthreads();
    if (s >= d.nsweeps) return;
    const int K = sweep_steps(d.n, d.w, s);
    const int Kp = (s > 0) ? sweep_steps(d.n, d.w, s - 1) : 0;
    bool kept = false;  // blk holds the block below of the previous step
    int have = 0;       // progress of sweep s-1 this workgroup has waited for
    for (int k = 0; k < K; ++k) {
      // a step that loaded its block below has waited for min(k + 2, Kp)
      // steps already: the wait before the next step is then not repeated
      const int need = min(k + 2, Kp);
      if (s > 0 && have < need) {
        if (!wait_prev(d, sh, s, need)) return;
        have = need;
      }
      const int need_below = (s > 0) ? min(k + 3, Kp) : 0;
      const int st = sb2st_step(d, sh, s, k, kept && k >= 1, need_below);
      kept = (st & kS2Kept) != 0;
      if (kept) have = max(have, need_below);  // it waited before its block below
      if (st & kS2Published) {
        __syncthreads();  // the next step reads the block below that blk now holds
      } else {
        // a step that ended early: every thread's stores, then the progress word
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (!sh.go) return;  // the wait inside the step gave up
        if (tid == 0)
          __hip_atomic_store(d.progress + s, k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// AB(k, c) = A(c + k, c) for k <= w, zero for w < k <= 2w
__global__ void k_band_copy(const double *A, int64_t lda, int n, int w, double *AB, int64_t ldab) {
  const int64_t total = (int64_t)ldab * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx % ldab);
    const int64_t c = idx / ldab;
    double v = 0.0;
    if (k <= w && c + k < n) v = A[(c + k) + c * lda];
    AB[idx] = v;
  }
}

__global__ void k_tridiag_extract(const double *AB, int64_t ldab, int n, double *dg, double *e) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    dg[i] = AB[(int64_t)i * ldab];
    if (i < n - 1) e[i] = AB[1 + (int64_t)i * ldab];
  }
}

int launch_sb2st(const double *A, int64_t lda, int n, int w, double *AB, int64_t ldab,
                 unsigned *sweep_ctr, int *progress, int *flags, long long timeout_ticks, int nwg,
                 double *dg, double *e, hipStream_t s) {
  {
    const int64_t total = ldab * (int64_t)n;
    int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_band_copy, dim3(blocks), dim3(256), 0, s, A, lda, n, w, AB, ldab);
    BR_HIP_CHECK(hipGetLastError());
  }
  const int nsweeps = std::max(0, n - 2);
  if (w > 1 && nsweeps > 0) {
    Sb2stDesc dd{};
    dd.AB = AB; dd.ldab = ldab; dd.n = n; dd.w = w; dd.nsweeps = nsweeps;
    dd.sweep_ctr = sweep_ctr; dd.progress = progress;
    dd.status = flags; dd.abort_flag = flags + 1; dd.timeout_ticks = timeout_ticks;
    hipLaunchKernelGGL(k_sb2st, dim3(std::max(1, std::min(nwg, nsweeps))), dim3(kS2T), 0, s, dd);
    BR_HIP_CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_tridiag_extract, dim3(std::max(1, std::min(1024, (n + 255) / 256))),
                     dim3(256), 0, s, (const double *)AB, ldab, n, dg, e);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

// ---------------------------------------------------------------------------
// Eigenvalues of the tridiagonal matrix: multisection on Sturm counts.  A
// group of G lanes of a wave per eigenvalue index k: the lanes count the
// eigenvalues below G points spread evenly inside the current interval [a, b]
// (which holds eigenvalue k), and the interval shrinks to the subinterval
// where the count passes k, G + 1 times narrower per round, until a and b are
// adjacent doubles or within 2 eps of the matrix's Gershgorin scale.  The
// count is the number of negative pivots of LDL^T of T - x I (a zero pivot
// counts as -pivmin).  A wider section takes fewer rounds but more counts in
// all (G / log2(G+1) per bit of the result); G is the smallest that still
// gives the chip about two waves per SIMD.
// ---------------------------------------------------------------------------
__global__ void k_tridiag_bounds(const double *dg, const double *e, int n, double *bounds) {
  __shared__ double slo[256], shi[256], se2[256];
  const int t = threadIdx.x;
  double lo = 1e308, hi = -1e308, e2 = 0.0;
  for (int i = t; i < n; i += 256) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0);
    lo = fmin(lo, dg[i] - r);
    hi = fmax(hi, dg[i] + r);
    if (i < n - 1) e2 = fmax(e2, e[i] * e[i]);
  }
  slo[t] = lo; shi[t] = hi; se2[t] = e2;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) {
      slo[t] = fmin(slo[t], slo[t + off]);
      shi[t] = fmax(shi[t], shi[t + off]);
      se2[t] = fmax(se2[t], se2[t + off]);
    }
    __syncthreads();
  }
  if (t == 0) {
    const double pivmin = 2.2250738585072014e-308 * fmax(se2[0], 1.0);
    const double scale = fmax(fabs(slo[0]), fabs(shi[0]));
    const double pad = 4.0 * 2.220446049250313e-16 * scale + pivmin;
    bounds[0] = slo[0] - pad;
    bounds[1] = shi[0] + pad;
    bounds[2] = pivmin;
    bounds[3] = scale;
  }
}

// 1/x from the hardware approximation plus two Newton steps (each squares
// the relative error): a few units in the last place, and a much shorter
// dependence chain than a correctly rounded division, which sits on the
// Sturm recurrence's sequential chain.  A count from slightly perturbed
// pivots is the exact count of a tridiagonal matrix within a few ulps of
// the given one, as with any floating-point Sturm count.
__device__ __forceinline__ double s2_rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

template <int G>
__global__ __launch_bounds__(256) void k_tridiag_eig(const double *dg, const double *e, int n,
                                                     const double *bounds, double *lam) {
  const int lane = threadIdx.x & 63;
  const int j = lane % G, g0 = lane - j;  // this lane's point, its group's first lane
  const int k = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G);
  if (k >= n) return;  // whole groups (G divides 64)
  double a = bounds[0], b = bounds[1];
  const double pivmin = bounds[2];
  const double tol = 2.0 * 2.220446049250313e-16 * bounds[3];
  for (int round = 0; round < 64; ++round) {
    if (b - a <= tol) break;  // a and b are uniform in the group
    const double x = a + (b - a) * (double)(j + 1) * (1.0 / (G + 1));
    // Sturm count below x
    int cnt = 0;
    double q = dg[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
    for (int i = 1; i < n; ++i) {
      const double ei = e[i - 1];
      q = (dg[i] - x) - (ei * ei) * s2_rcp(q);
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += (q < 0.0);
    }
    // first point of the group whose count exceeds k: eigenvalue k lies below it
    const unsigned long long above = __ballot(cnt > k);
    const unsigned long long mine = (G == 64) ? above : (above >> g0) & ((1ull << (G & 63)) - 1);
    const int f = mine ? __builtin_ctzll(mine) : G;
    const double xf = __shfl(x, g0 + (f < G ? f : G - 1));
    const double xp = __shfl(x, g0 + (f > 0 ? f - 1 : 0));
    const double na = (f > 0) ? xp : a;
    const double nb = (f < G) ? xf : b;
    if (na == a && nb == b) break;  // no progress: a and b (nearly) adjacent
    a = na;
    b = nb;
  }
  if (j == 0) lam[k] = 0.5 * (a + b);
}

int launch_tridiag_eig(const double *dg, const double *e, int n, double *bounds, double *lam,
                       hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_tridiag_bounds, dim3(1), dim3(256), 0, s, dg, e, n, bounds);
  BR_HIP_CHECK(hipGetLastError());
  // lanes per eigenvalue: about two waves per SIMD of 256 CUs from n G lanes
  // (measured at n = 16384 and 8192: one wave per SIMD leaves the counts'
  // latency exposed, four make the wider sections' extra counts cost more)
  const int G = (n >= 16384) ? 8 : (n >= 8192) ? 16 : (n >= 4096) ? 32 : 64;
  const int64_t threads = (int64_t)n * G;
  const dim3 grid((unsigned)((threads + 255) / 256));
  const double *bd = bounds;
  if (G == 8) hipLaunchKernelGGL(k_tridiag_eig<8>, grid, dim3(256), 0, s, dg, e, n, bd, lam);
  else if (G == 16) hipLaunchKernelGGL(k_tridiag_eig<16>, grid, dim3(256), 0, s, dg, e, n, bd, lam);
  else if (G == 32) hipLaunchKernelGGL(k_tridiag_eig<32>, grid, dim3(256), 0, s, dg, e, n, bd, lam);
  else hipLaunchKernelGGL(k_tridiag_eig<64>, grid, dim3(256), 0, s, dg, e, n, bd, lam);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace br
