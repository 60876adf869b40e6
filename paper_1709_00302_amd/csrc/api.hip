// api.hip -- C ABI, workspace and the blocked drivers of the band reductions.
//
// SY2SB driver (Sec. 2.1; look-ahead Variant V2 of Sec. 2.2 when 2b > w and
// the V1 partition when 2b <= w).  Per panel c (width pb, r = c + w,
// j = n - r):
//   1. panel QR of A0 = A[r:n, c:c+pb] -> V (explicit), tau, T, in-place R/v
//      (eq. updateA0; CholeskyQR2 + Householder reconstruction, recon.hip)
//   2. Wt = V T                          (the paper's W = -Wt, Sec. 4.1)
//   3. A1 -= V T^T (V^T A1) = V (Wt^T A1) on the w-pb in-band columns right
//      of the panel (eq. updateA1; empty when b = w)
//   4. X = A2 Wt (SYMM)                  (eq. updateA2symm)
//   5. M = Wt^T X, W = X - 1/2 V M       (eqs. updateA2gemm1/gemm2, X3 = -W)
//   6. A2 -= W V^T + V W^T (SYR2K, lower triangle; eq. updateA2syr2k)
// Look-ahead (Sec. 2.2) factors the next panel (steps 1-2) on a second stream:
// Variant V1 (the next panel lies in A1, 2b <= w) forks right after step 3;
// Variant V2 (2b > w) first applies step 6 to the columns of A2 that belong to
// the next panel (A2^L), forks, and applies the rest (A2^R) meanwhile.
//
// GE2GB driver (Sec. 3.1, triangular-band form, b <= w).  Per block c:
//   1. left QR of A[c:m, c:c+pb], Wtq = V Tq      (eq. updateB)
//   2. E = A[c:m, c+pb:n]: E -= V (Wtq^T E)        (eq. updateCD)
//   3. right LQ of A[c:c+pr, c+w:n], Wtp = U Tp   (eq. updateC)
//   4. D = A[c+pr:m, c+w:n]: D -= (D Wtp) U^T      (eq. updateD)
#include <mutex>
#include <algorithm>
#include <vector>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "common.hpp"

namespace br {

int hip_fail(hipError_t e, const char *what) {
  if (getenv("BANDRED_VERBOSE")) fprintf(stderr, "bandred: %s failed: %s\n", what, hipGetErrorString(e));
  return BANDRED_ERR_HIP;
}

// ---------------------------------------------------------------------------
// profiling (optional): events around every launch
// ---------------------------------------------------------------------------
enum Cls { C_PANEL = 0, C_LARFT, C_SYMM, C_SYR2K, C_GEMM_SMALL, C_REDUCE, C_GEMM_UPD,
           C_PANEL_SMALL, C_OTHER, C_BATCHED, C_NCLS };
static const char *kClsNames[C_NCLS] = {"panel_qr", "larft", "symm", "syr2k", "gemm_small",
                                        "reduce", "gemm_update", "panel_small", "other",
                                        "batched"};
struct ProfRec {
  int cls;
  double flops;
  hipEvent_t a, b;
};
static bool g_prof = false;
static std::vector<ProfRec> g_prof_recs;
static std::vector<hipEvent_t> g_ev_pool;

static hipEvent_t ev_get() {
  if (!g_ev_pool.empty()) {
    hipEvent_t e = g_ev_pool.back();
    g_ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct ProfScope {
  ProfRec rec;
  hipStream_t s;
  bool on;
  ProfScope(int cls, double flops, hipStream_t st) : s(st), on(g_prof) {
    if (!on) return;
    rec.cls = cls;
    rec.flops = flops;
    rec.a = ev_get();
    rec.b = ev_get();
    if (rec.a) hipEventRecord(rec.a, s);
  }
  ~ProfScope() {
    if (!on) return;
    if (rec.b) hipEventRecord(rec.b, s);
    if (rec.a && rec.b) g_prof_recs.push_back(rec);
  }
};

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------

// A device table of one batched call's matrices.  A table that a captured
// HIP graph has used is never rewritten or freed (the graph keeps its device
// address); other tables are reused for later uploads.
struct BatchTable {
  std::vector<BatchEntry> host;  // content (sorted as uploaded)
  BatchEntry *dev = nullptr;
  size_t cap = 0;                // entries dev holds
  bool captured = false;
};

struct DevState {
  bool props = false;         // device properties read (no allocation)
  bool init = false;          // streams, events and the status words created
  int num_cu = 0;
  long long timeout_ticks = 0;
  long long default_ticks = 0;
  char *base = nullptr;
  size_t bytes = 0;
  bool base_captured = false; // a captured graph refers to base
  std::vector<void *> retired;// workspaces a captured graph may still use
  hipEvent_t done = nullptr;  // completion of the previous call's work
  hipStream_t aux = nullptr;  // look-ahead (panel) stream
  hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_c = nullptr, ev_d = nullptr;
  hipEvent_t ev_h = nullptr;  // head of a look-ahead panel (see panel_factor)
  int *flags = nullptr;       // [0] status, [1] abort   (device)
  // batched calls: uploaded matrix tables, a pinned staging copy, the work
  // counter and the per-workgroup scratch
  std::vector<BatchTable> tables;
  BatchEntry *bt_stage = nullptr;
  size_t bt_stage_cap = 0;
  hipEvent_t bt_ev = nullptr; // completion of the last upload from the staging copy
  unsigned *bt_queue = nullptr;
  double *bt_ws = nullptr;
  int bt_wgs = 0;             // workgroups bt_ws holds
  bool bt_ws_captured = false;
};
static std::mutex g_mu;
static DevState g_dev[64];
// status words of the most recent call on each device (the library's own, or
// those inside the no-allocation scratch)
static int *g_last_flags[64];

// Device properties only: no stream, event or memory is created.
static int dev_props(DevState &st, int dev) {
  if (st.props) return 0;
  hipDeviceProp_t prop;
  BR_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return BANDRED_ERR_UNSUPPORTED;
  st.num_cu = prop.multiProcessorCount;
  int rate_khz = 0;
  BR_HIP_CHECK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
  if (rate_khz <= 0) rate_khz = 100000;
  st.default_ticks = (long long)rate_khz * 1000LL * 10LL;  // 10 s per wait
  if (st.timeout_ticks <= 0) st.timeout_ticks = st.default_ticks;
  st.props = true;
  return 0;
}

static int current_device(int *dev) {
  BR_HIP_CHECK(hipGetDevice(dev));
  if (*dev < 0 || *dev >= 64) return BANDRED_ERR_UNSUPPORTED;
  return 0;
}

// index of the current device (valid once dev_state or dev_props succeeded)
static int current_dev_index() {
  int dev = 0;
  return current_device(&dev) == 0 ? dev : 0;
}

static int dev_state(DevState **out) {
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  DevState &st = g_dev[dev];
  rc = dev_props(st, dev);
  if (rc) return rc;
  if (!st.init) {
    BR_HIP_CHECK(hipEventCreateWithFlags(&st.done, hipEventDisableTiming));
    BR_HIP_CHECK(hipEventCreateWithFlags(&st.ev_a, hipEventDisableTiming));
    BR_HIP_CHECK(hipEventCreateWithFlags(&st.ev_b, hipEventDisableTiming));
    BR_HIP_CHECK(hipEventCreateWithFlags(&st.ev_c, hipEventDisableTiming));
    BR_HIP_CHECK(hipEventCreateWithFlags(&st.ev_d, hipEventDisableTiming));
    BR_HIP_CHECK(hipEventCreateWithFlags(&st.ev_h, hipEventDisableTiming));
    BR_HIP_CHECK(hipStreamCreateWithFlags(&st.aux, hipStreamNonBlocking));
    BR_HIP_CHECK(hipMalloc((void **)&st.flags, 64));
    BR_HIP_CHECK(hipMemset(st.flags, 0, 64));
    BR_HIP_CHECK(hipEventRecord(st.done, st.aux));
    BR_HIP_CHECK(hipEventCreateWithFlags(&st.bt_ev, hipEventDisableTiming));
    BR_HIP_CHECK(hipEventRecord(st.bt_ev, st.aux));
    BR_HIP_CHECK(hipMalloc((void **)&st.bt_queue, 256));
    BR_HIP_CHECK(hipDeviceSynchronize());
    st.init = true;
  }
  *out = &st;
  return 0;
}

// Grow the workspace to at least `bytes`; waits for the previous call first.
// A workspace that a captured HIP graph refers to is retired, not freed: a
// replay of that graph after this call still finds its memory.
static int ws_reserve(DevState &st, size_t bytes) {
  if (bytes <= st.bytes) return 0;
  BR_HIP_CHECK(hipEventSynchronize(st.done));
  if (st.base) {
    if (st.base_captured) st.retired.push_back(st.base);
    else BR_HIP_CHECK(hipFree(st.base));
  }
  st.base = nullptr;
  st.bytes = 0;
  st.base_captured = false;
  const size_t want = bytes + (bytes >> 3);
  if (hipMalloc((void **)&st.base, want) != hipSuccess) {
    (void)hipGetLastError();
    st.base = nullptr;
    return BANDRED_ERR_ALLOC;
  }
  st.bytes = want;
  return 0;
}

// Stream capture (HIP graphs): a call recorded into a graph may not allocate
// (the workspace must already be reserved by an earlier eager call at least
// as large), skips the wait on and the record of the cross-call completion
// event (the caller orders replays against other calls), and runs without
// the profiling events.  The workspace is then marked as referenced by a
// graph (see ws_reserve).
static int capture_check(hipStream_t s, size_t need, DevState &st, bool *capturing) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  BR_HIP_CHECK(hipStreamIsCapturing(s, &cap));
  *capturing = cap != hipStreamCaptureStatusNone;
  if (*capturing && (g_prof || need > st.bytes)) return BANDRED_ERR_UNSUPPORTED;
  if (*capturing) st.base_captured = true;
  return 0;
}

struct Arena {
  char *p;
  size_t off = 0;
  explicit Arena(char *base) : p(base) {}
  template <class T>
  T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *r = reinterpret_cast<T *>(p + off);
    off += count * sizeof(T);
    return r;
  }
};

static size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// GEMM helpers
// ---------------------------------------------------------------------------
struct Ctx {
  DevState *st;
  hipStream_t s;
  double *part;
  size_t part_cap;  // doubles
  char *oz = nullptr;  // digit planes of the exact-split products (P_OZ)
  size_t oz_cap = 0;   // bytes
  int max_chunks = 0;  // bandred_opts_t.update_chunks (0: the defaults below)
  int lds_cap = 0;     // bandred_opts_t.update_lds_cap
  // exact split, SY2SB: the SYR2K records the row maxima of the next
  // trailing matrix (indices >= oz_rec_off of the current one) into oz_rec,
  // and the next SYMM slices its symmetric operand with them (oz_rmax_in)
  unsigned long long *oz_rec = nullptr;
  int oz_rec_off = 0;
  const unsigned long long *oz_rmax_in = nullptr;
};

// ---------------------------------------------------------------------------
// exact-split products (P_OZ, ozaki.hip)
// ---------------------------------------------------------------------------
// bytes of one product's slices: row maxima and exponents (two segments at
// most) and the digit planes of op(A) (M rows) and op(B) (N columns) over K
// (each segment padded to a multiple of 64)
static size_t oz_need(int64_t M, int64_t N, int64_t K) {
  const size_t Kp = round_up((size_t)K, 64) + 64;
  const size_t rows = round_up((size_t)M, 64) + round_up((size_t)N, 64);  // 64-row blocks
  return 6 * 256 + 24 * (size_t)(M + N) + (size_t)kOzS * rows * Kp;
}
// bound over the products of a driver whose dimensions are at most L1, L2
// (the matrix) and s2 (a block of reflectors), in any roles
static size_t oz_bound(int64_t L1, int64_t L2, int64_t s2) {
  const int64_t d[3] = {L1, L2, s2};
  size_t m = 0;
  for (int k = 0; k < 3; ++k)  // d[k] is the inner dimension
    m = std::max(m, oz_need(d[(k + 1) % 3], d[(k + 2) % 3], d[k]));
  return round_up(m, 256);
}

// C = alpha op(A) op(B) + beta C (E_AXPBY), or C -= op(A) op(B) on the lower
// triangle of columns [c0, c1) (E_SYR2K), through int8 digit planes.  A rank-2k
// update [P | Q] [R | S]^T passes ks = the width of P: the two halves of the
// inner dimension get scales of their own.
static int gemm_oz(Ctx &cx, int cls, int opa, int opb, int epi, int M, int N, int K, int ks,
                   const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                   int64_t ldc, double alpha, double beta, int rot, int c0, int c1, double flops,
                   hipStream_t s) {
  const int rec_off = cx.oz_rec_off - c0;  // (in the coordinates from (c0, c0))
  if (epi == E_SYR2K) {
    // the rows [c0, M) of op(A) and the columns [c0, c1) of op(B) only (the
    // tiles then start on the 64-row blocks of their planes): C from (c0, c0)
    if (c1 <= c0 || M <= c0) return 0;
    A += c0;  // op(A) = A_N: row r at A[r + k lda]
    B += c0;  // op(B) = B_TROT: column c at B[c + kr ldb]
    C += c0 + (int64_t)c0 * ldc;
    M -= c0;
    N = c1 - c0;
    c1 = N;
    c0 = 0;
  }
  if (!cx.oz || oz_need(M, N, K) > cx.oz_cap) return BANDRED_ERR_UNSUPPORTED;
  int L0 = 0;
  const int Kp = oz_plane_cols(K, ks, &L0);
  Arena ar(cx.oz);
  unsigned long long *mxa = ar.take<unsigned long long>(2 * (size_t)M);
  unsigned long long *mxb = ar.take<unsigned long long>(2 * (size_t)N);
  int *ea = ar.take<int>(2 * (size_t)M), *eb = ar.take<int>(2 * (size_t)N);
  int8_t *PA = ar.take<int8_t>((size_t)kOzS * round_up((size_t)M, 64) * Kp);
  int8_t *PB = ar.take<int8_t>((size_t)kOzS * round_up((size_t)N, 64) * Kp);
  const int *abort = cx.st->flags + 1;
  ProfScope ps(cls, flops, s);
  int rc = oz_slice(A, lda, opa, M, K, ks, 0, 0, mxa, ea, PA, s,
                    opa == A_SYM ? cx.oz_rmax_in : nullptr);
  if (rc) return rc;
  rc = oz_slice(B, ldb, opb, N, K, ks, rot, 1, mxb, eb, PB, s);
  if (rc) return rc;
  if (epi == E_SYR2K)
    return oz_gemm(E_SYR2K, PA, PB, ea, eb, M, N, Kp, L0, 1, Kp, C, ldc, 1.0, 0.0, nullptr, c0,
                   c1, abort, s, cx.oz_rec, rec_off);
  // two 64 x 64 workgroups per CU are resident: split k when the tiles do
  // not fill the chip (chunks of at least 256, partial sums within the buffer)
  const int64_t tiles = (int64_t)((M + 63) / 64) * ((N + 63) / 64);
  const int64_t slots = 2 * (int64_t)cx.st->num_cu;
  int nk = 1;
  if (tiles < slots && Kp >= 512) {
    nk = (int)std::min<int64_t>((2 * slots + tiles - 1) / tiles, Kp / 256);
    while (nk > 1 && (size_t)nk * M * N > cx.part_cap) --nk;
  }
  if (nk <= 1)
    return oz_gemm(E_AXPBY, PA, PB, ea, eb, M, N, Kp, L0, 1, Kp, C, ldc, alpha, beta, nullptr, 0,
                   0, abort, s);
  const int kchunk = (int)round_up((size_t)(Kp + nk - 1) / nk, 64);
  nk = (Kp + kchunk - 1) / kchunk;
  rc = oz_gemm(E_PART, PA, PB, ea, eb, M, N, Kp, L0, nk, kchunk, nullptr, 0, 1.0, 0.0, cx.part,
               0, 0, abort, s);
  if (rc) return rc;
  return launch_reduce_partials(cx.part, nk, M, N, alpha, C, ldc, beta, s, nullptr, 0, abort);
}

// C(M x N) = alpha op(A) op(B) + beta C, split over k when that fills the chip.
static int gemm(Ctx &cx, int cls, int opa, int opb, int prec, int M, int N, int K,
                const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                int64_t ldc, double alpha, double beta, hipStream_t s,
                const int *gate = nullptr, int gate_val = 0, double *C2 = nullptr,
                int64_t ldc2 = 0, int c2_trans = 0, int lds_pad = 0, int kseg = 0) {
  if (M <= 0 || N <= 0) return 0;
  if (K <= 0) {
    if (beta == 1.0) return 0;
    return BANDRED_ERR_UNSUPPORTED;  // never needed by the drivers
  }
  if (prec == P_OZ) {
    if (gate || C2) return BANDRED_ERR_UNSUPPORTED;  // (only FP64 products use these)
    return gemm_oz(cx, cls, opa, opb, E_AXPBY, M, N, K, kseg, A, lda, B, ldb, C, ldc, alpha, beta,
                   0, 0, 0, 2.0 * M * N * (double)K, s);
  }
  GemmDesc d{};
  d.M = M; d.N = N; d.K = K;
  d.A = A; d.lda = lda; d.B = B; d.ldb = ldb; d.C = C; d.ldc = ldc;
  d.alpha = alpha; d.beta = beta;
  d.gate = gate; d.gate_val = gate_val;
  d.C2 = C2; d.ldc2 = ldc2; d.c2_trans = c2_trans;
  d.lds_pad = lds_pad;
  d.abort = cx.st->flags + 1;
  d.prio = (cls == C_PANEL || cls == C_GEMM_SMALL) ? 1 : 0;
  int tm = 128, tn = 128;
  gemm_tile_shape(E_AXPBY, M, N, 0, &tm, &tn);
  if (tm == 64 && tn == 64 && (M > 64 || N > 64)) tm = tn = 128;  // (may still take 64 x 64 below)
  const int tiles = ((M + tm - 1) / tm) * ((N + tn - 1) / tn);
  // workgroups resident at once: two per CU for the 128 x 128 tiles (VGPRs
  // and LDS), three for 128 x 64 and 64 x 128 (LDS), four for 64 x 64
  const int per_cu = (tm == 128 && tn == 128) ? 2 : (tm == 64 && tn == 64) ? 4 : 3;
  const int slots = per_cu * cx.st->num_cu;
  // k-chunk granularity: the panel's Gram products (beside the running update
  // more, shorter workgroups finish sooner) take chunks of 128 rows, or of 64
  // for outputs of one 64 x 64 tile (b <= 64), which need more splits to fill
  // the chip
  const int kg = (cls == C_PANEL && M <= 64 && N <= 64) ? 64 : 128;
  int ks = 1;
  if (tiles < slots && K > 512 && !C2) {  // (the second output needs a single pass)
    // split k so that the work runs in as few full rounds of resident
    // workgroups as possible: the time goes as rounds x (k chunk), plus the
    // reduction of the partial sums (memory bound, about one k unit per
    // 2.5e6 elements of each partial)
    const int maxks = K / (cls == C_PANEL ? kg : 256);  // (kg = 128 or 64 for the panel)
    double best = 0.0;
    for (int c = 1; c <= maxks; ++c) {
      if ((size_t)c * M * N > cx.part_cap) break;
      const int kc = (int)round_up((K + c - 1) / c, kg);
      const int kk = (K + kc - 1) / kc;
      const int rounds = (tiles * kk + slots - 1) / slots;
      const double cost =
          (double)rounds * kc + (kk > 1 ? (kk + 1) * ((double)M * N / 2.5e6) : 0.0);
      if (c == 1 || cost < best - 1e-9) {
        best = cost;
        ks = kk;
      }
    }
  }
  const double flops = 2.0 * M * N * (double)K;
  if (ks == 1) {
    // too few 128 x 128 tiles to occupy every CU and no k split: 64 x 64
    // tiles give four times the workgroups
    if (tm == 128 && tn == 128 && tiles < cx.st->num_cu) d.tile64 = 1;
    d.kchunk = (int)round_up(K, kBK);
    ProfScope ps(cls, flops, s);
    return launch_gemm(opa, opb, E_AXPBY, prec, d, 1, s);
  }
  d.kchunk = (int)round_up((K + ks - 1) / ks, kg);
  ks = (K + d.kchunk - 1) / d.kchunk;
  d.part = cx.part;
  {
    ProfScope ps(cls, flops, s);
    int rc = launch_gemm(opa, opb, E_PART, prec, d, ks, s);
    if (rc) return rc;
  }
  ProfScope ps(C_REDUCE, 0.0, s);
  return launch_reduce_partials(cx.part, ks, M, N, alpha, C, ldc, beta, s, gate, gate_val,
                                cx.st->flags + 1);
}

// A2(lower, columns [c0, c1)) -= W V^T + V W^T with WV = [W | V] (j x 2pb).
static int syr2k(Ctx &cx, int prec, int j, int pb, const double *WV, int64_t ldwv, double *A2,
                 int64_t lda, int c0, int c1, hipStream_t s, int lds_pad = 0) {
  if (c1 <= c0) return 0;
  if (prec == P_OZ) {
    const double r0 = (double)(j - c0), r1 = (double)(j - c1);
    return gemm_oz(cx, C_SYR2K, A_N, B_TROT, E_SYR2K, j, j, 2 * pb, pb, WV, ldwv, WV, ldwv, A2,
                   lda, 1.0, 0.0, pb, c0, c1, 2.0 * pb * (r0 * (r0 + 1) - r1 * (r1 + 1)), s);
  }
  GemmDesc d{};
  d.lds_pad = lds_pad;
  d.abort = cx.st->flags + 1;
  d.M = j; d.N = j; d.K = 2 * pb;
  d.A = WV; d.lda = ldwv; d.B = WV; d.ldb = ldwv;
  d.C = A2; d.ldc = lda;
  d.rot = pb; d.c0 = c0; d.c1 = c1;
  d.kchunk = 2 * pb;
  {  // lower tiles of 128 x 128 in the column range; 64 x 64 below one per CU
    const int nI = (j - c0 + 127) / 128, nJ = (c1 - c0 + 127) / 128;
    const int64_t lower = (int64_t)nJ * nI - (int64_t)nJ * (nJ - 1) / 2;
    if (lower < cx.st->num_cu) d.tile64 = 1;
  }
  // lower-trapezoid flops of the column range
  const double rows0 = (double)(j - c0), rows1 = (double)(j - c1);
  const double elems = 0.5 * (rows0 * (rows0 + 1) - rows1 * (rows1 + 1));
  ProfScope ps(C_SYR2K, 2.0 * 2.0 * pb * elems, s);
  return launch_gemm(A_N, B_TROT, E_SYR2K, prec, d, 1, s);
}

// Trailing updates that run beside a panel factorisation are issued as a few
// consecutive launches over column chunks instead of one.  The single-workgroup
// b x b kernels of the panel need a whole CU, which a running update never
// frees (a finished workgroup's slot is refilled at once); between two launches
// on one stream the CUs drain, and a waiting panel kernel takes one.  At most
// three chunks (two drains for the panel's three such kernels: fewer chunks
// leave them waiting longer, more add launch tails that cost more than they
// save), each at least two full rounds of resident 128 x 128 workgroups.
// Every element is still computed by one tile in the same order.  The SYR2K
// takes at most two (its upper tiles exit early, so CUs drain within a launch
// too; measured on SY2SB n=16384: 158.8 ms with two, 160.1 with three).
constexpr int kMaxChunks = 3;
constexpr int kMaxSyr2kChunks = 2;
// Below a trailing order (GE2GB: update rows) of 8192 the panel beside the
// update is the longer of the two by a wider margin; there the update's
// launches reserve 20 KB of extra LDS per workgroup, which leaves one of its
// 128 x 128 workgroups per CU (86 KB of 160) and the rest of the CU to the
// panel's kernels that fit beside one (measured: SY2SB n=8192 w=64 1.3%
// faster, n=16384 w=128 0.5%, GE2GB 8192^2 w=64 1.2%; applied at every order
// the cap costs the large updates more than it gains).
constexpr int kUpdateCapBelow = 8192;
constexpr int kUpdateCapLds = 20 * 1024;
static int update_chunks(const DevState *st, int64_t tiles128, int maxc) {
  const int64_t per = 4 * (int64_t)st->num_cu;  // two rounds of two workgroups per CU
  return (int)std::max<int64_t>(1, std::min<int64_t>(maxc, tiles128 / per));
}
// extra LDS of an update launch beside a panel, for an update of `rows` rows
static int update_lds_pad(const Ctx &cx, int64_t rows) {
  if (cx.lds_cap == 1) return kUpdateCapLds;
  if (cx.lds_cap == 2) return 0;
  return rows <= kUpdateCapBelow ? kUpdateCapLds : 0;
}

// syr2k over columns [c0, c1) as update_chunks() launches of about equal
// lower-trapezoid area, boundaries on 128-column tiles.
static int syr2k_chunked(Ctx &cx, int prec, int j, int pb, const double *WV, int64_t ldwv,
                         double *A2, int64_t lda, int c0, int c1, hipStream_t s) {
  if (c1 <= c0) return 0;
  const int64_t nI = (j - c0 + 127) / 128, nJ = (c1 - c0 + 127) / 128;
  const int nck = update_chunks(cx.st, nJ * nI - nJ * (nJ - 1) / 2,
                                cx.max_chunks > 0 ? cx.max_chunks : kMaxSyr2kChunks);
  auto area = [&](double x) {  // lower-trapezoid elements of columns [c0, x)
    const double r0 = j - c0, r1 = j - x;
    return 0.5 * (r0 * (r0 + 1) - r1 * (r1 + 1));
  };
  const double tot = area(c1);
  int lo = c0;
  for (int k = 1; k <= nck; ++k) {
    int hi = c1;
    if (k < nck) {
      // smallest tile boundary whose area reaches k / nck of the total
      hi = lo;
      while (hi < c1 && area(hi) < tot * k / nck) hi = std::min(c1, hi + 128);
    }
    int rc = syr2k(cx, prec, j, pb, WV, ldwv, A2, lda, lo, hi, s, update_lds_pad(cx, j));
    if (rc) return rc;
    lo = hi;
  }
  return 0;
}

// C(M x N) = alpha op(A) op(B) + beta C with K <= 512 (no k split) as
// update_chunks() launches over column chunks of 128-multiples.
static int gemm_chunked(Ctx &cx, int cls, int opa, int opb, int prec, int M, int N, int K,
                        const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                        int64_t ldc, double alpha, double beta, hipStream_t s, int kseg = 0) {
  const int64_t tiles = (int64_t)((M + 127) / 128) * ((N + 127) / 128);
  const int nck =
      (K <= 512) ? update_chunks(cx.st, tiles, cx.max_chunks > 0 ? cx.max_chunks : kMaxChunks) : 1;
  const int nt = (N + 127) / 128;
  for (int k = 0, n0 = 0; k < nck && n0 < N; ++k) {
    const int n1 = (k == nck - 1) ? N : std::min(N, 128 * (int)((int64_t)nt * (k + 1) / nck));
    if (n1 <= n0) continue;
    const double *Bk = (opb == B_N) ? B + (int64_t)n0 * ldb : B + n0;
    int rc = gemm(cx, cls, opa, opb, prec, M, n1 - n0, K, A, lda, Bk, ldb,
                  C + (int64_t)n0 * ldc, ldc, alpha, beta, s, nullptr, 0, nullptr, 0, 0,
                  update_lds_pad(cx, M), kseg);
    if (rc) return rc;
    n0 = n1;
  }
  return 0;
}

// Scratch of one panel factorisation.
struct PanelWs {
  double *G, *G2, *R1, *R1i, *R2, *R2i, *Qtop, *Ui, *M, *Rh0, *S, *sgn, *Q1;
  double *part2, *piv;
  static size_t bytes(int mmax, int b) {
    return 256 * 16 + 8 * ((size_t)11 * b * b + (size_t)b + (size_t)mmax * b +
                           (size_t)2 * 256 * kNbMax + (size_t)kNbMax * kNbMax);
  }
  void carve(Arena &ar, int mmax, int b) {
    const size_t bb = (size_t)b * b;
    G = ar.take<double>(bb); G2 = ar.take<double>(bb);
    R1 = ar.take<double>(bb); R1i = ar.take<double>(bb);
    R2 = ar.take<double>(bb); R2i = ar.take<double>(bb);
    Qtop = ar.take<double>(bb); Ui = ar.take<double>(bb);
    M = ar.take<double>(bb); Rh0 = ar.take<double>(bb); S = ar.take<double>(bb);
    sgn = ar.take<double>(b);
    Q1 = ar.take<double>((size_t)mmax * b);
    part2 = ar.take<double>((size_t)2 * 256 * kNbMax);
    piv = ar.take<double>((size_t)kNbMax * kNbMax);
  }
};

// The per-column kernel (exact Householder, one grid barrier per column).
static int panel_columns(Ctx &cx, bool rowmajor, double *P, int64_t ldp, int m, int nb, double *V,
                         int64_t ldv, double *tau, PanelWs &pw, unsigned *counter, int panel_rows,
                         const int *gate, int gate_val, hipStream_t s) {
  DevState &st = *cx.st;
  const int LDW = (nb & 1) ? nb : nb + 1;
  const int rmax = (150 * 1024) / (LDW * 8);
  int R = panel_rows > 0 ? panel_rows : 128;
  if (R < nb) R = nb;
  int maxwg = st.num_cu - 16;
  if (maxwg > 240) maxwg = 240;
  if ((m + R - 1) / R > maxwg) R = (m + maxwg - 1) / maxwg;
  if (R > rmax) return BANDRED_ERR_UNSUPPORTED;
  const int nwg = (m + R - 1) / R;
  PanelDesc d{};
  d.P = P; d.ldp = ldp; d.m = m; d.nb = nb; d.R = R;
  d.V = V; d.ldv = ldv; d.tau = tau;
  d.part = pw.part2; d.piv = pw.piv; d.counter = counter;
  d.status = st.flags; d.abort_flag = st.flags + 1;
  d.timeout_ticks = st.timeout_ticks;
  d.gate = gate; d.gate_val = gate_val;
  ProfScope ps(C_PANEL, 2.0 * (double)m * nb * nb, s);
  return launch_panel(rowmajor, d, nwg, s);
}

// Factor the m x nb panel P (column panel, or row panel when rowmajor):
// in-place R / v storage, explicit V (m x nb, ld ldv), tau and T (nb x nb).
//   method 1: per-column kernel + S = V^T V + T recurrence.
//   method 0/2: CholeskyQR2 + Householder reconstruction; if the first
//   Cholesky flags the panel (rank deficient, or a column that is zero below
//   its diagonal by the panel's structure), the per-column path runs instead
//   (all kernels are gated on the device flag, no host round trip).
static int panel_factor(Ctx &cx, bool rowmajor, double *P, int64_t ldp, int m, int nb, double *V,
                        int64_t ldv, double *tau, double *T, int ldt, PanelWs &pw,
                        unsigned *counter, int *flag, int *structure, int method, int panel_rows,
                        hipStream_t s, hipEvent_t head_ev = nullptr, int head_at = 0,
                        bool *head_done = nullptr) {
  // head_ev (optional) is recorded on s at point head_at of the CholeskyQR2
  // path: 1 after the first Gram product, 2 after the first Cholesky and
  // inverse, 3 after the second Gram product, 4 after the second Cholesky
  int rc;
  auto head = [&](int at) -> int {
    if (head_ev && head_at == at) {
      BR_HIP_CHECK(hipEventRecord(head_ev, s));
      if (head_done) *head_done = true;
    }
    return 0;
  };
  // a square panel's last column has no rows below the diagonal (tau = 0 by
  // the Householder convention): factor it column by column
  if (m <= nb) method = 1;
  if (method == 1) {
    rc = panel_columns(cx, rowmajor, P, ldp, m, nb, V, ldv, tau, pw, counter, panel_rows, nullptr,
                       0, s);
    if (rc) return rc;
    rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, P_F64, nb, nb, m, V, ldv, V, ldv, pw.S, nb, 1.0, 0.0, s);
    if (rc) return rc;
    ProfScope p2(C_LARFT, 0.0, s);
    return launch_larft(pw.S, nb, tau, nb, T, ldt, s);
  }
  const double flops = 2.0 * (double)m * nb * nb;
  rc = launch_panel_structure(P, ldp, rowmajor ? 1 : 0, m, nb, structure, s);
  if (rc) return rc;
  // G = P^T P ; R1 = chol(G), R1^-1
  rc = gemm(cx, C_PANEL, rowmajor ? A_N : A_T, rowmajor ? B_T : B_N, P_F64, nb, nb, m, P, ldp, P,
            ldp, pw.G, nb, 1.0, 0.0, s);
  if (rc) return rc;
  rc = head(1);
  if (rc) return rc;
  {
    ProfScope p2(C_PANEL_SMALL, 0.0, s);
    rc = launch_chol_inv(pw.G, nb, nb, 1e-10, pw.R1, pw.R1i, flag, structure, s);
    if (rc) return rc;
  }
  rc = head(2);
  if (rc) return rc;
  // Q1 = P R1^-1 ; G2 = Q1^T Q1 ; R2 = chol(G2), R2^-1
  rc = gemm(cx, C_PANEL, rowmajor ? A_T : A_N, B_N, P_F64, m, nb, nb, P, ldp, pw.R1i, nb, pw.Q1,
            m, 1.0, 0.0, s, flag, 0);
  if (rc) return rc;
  rc = gemm(cx, C_PANEL, A_T, B_N, P_F64, nb, nb, m, pw.Q1, m, pw.Q1, m, pw.G2, nb, 1.0, 0.0, s,
            flag, 0);
  if (rc) return rc;
  rc = head(3);
  if (rc) return rc;
  {
    ProfScope p2(C_PANEL_SMALL, 0.0, s);
    rc = launch_chol_inv(pw.G2, nb, nb, 1e-6, pw.R2, pw.R2i, flag, nullptr, s);
    if (rc) return rc;
  }
  rc = head(4);
  if (rc) return rc;
  // Qtop = Q1(0:nb, :) R2^-1 ; LU with signs, T, U^-1
  rc = gemm(cx, C_PANEL, A_N, B_N, P_F64, nb, nb, nb, pw.Q1, m, pw.R2i, nb, pw.Qtop, nb, 1.0, 0.0,
            s, flag, 0);
  if (rc) return rc;
  {
    ProfScope p2(C_PANEL_SMALL, 0.0, s);
    rc = launch_recon(pw.Qtop, nb, nb, V, ldv, T, ldt, tau, pw.Ui, pw.sgn, pw.piv, flag, s);
    if (rc) return rc;
  }
  // M = R2^-1 U^-1 ; Rh0 = R2 R1 ; V(nb:m, :) = Q1(nb:m, :) M ; write in place
  rc = gemm(cx, C_PANEL, A_N, B_N, P_F64, nb, nb, nb, pw.R2i, nb, pw.Ui, nb, pw.M, nb, 1.0, 0.0, s,
            flag, 0);
  if (rc) return rc;
  rc = gemm(cx, C_PANEL, A_N, B_N, P_F64, nb, nb, nb, pw.R2, nb, pw.R1, nb, pw.Rh0, nb, 1.0, 0.0,
            s, flag, 0);
  if (rc) return rc;
  if (m > nb) {
    // rows nb.. of the factored panel are those of V: the product stores them
    // to the panel as well (in place, transposed for a row panel), so the
    // finalisation below only writes the top nb x nb block
    rc = gemm(cx, C_PANEL, A_N, B_N, P_F64, m - nb, nb, nb, pw.Q1 + nb, m, pw.M, nb, V + nb, ldv,
              1.0, 0.0, s, flag, 0, rowmajor ? P + (int64_t)nb * ldp : P + nb, ldp,
              rowmajor ? 1 : 0);
    if (rc) return rc;
  }
  {
    ProfScope p2(C_PANEL_SMALL, flops, s);
    rc = launch_panel_finalize(P, ldp, rowmajor ? 1 : 0, std::min(m, nb), nb, V, ldv, pw.Rh0,
                               pw.sgn, flag, s);
    if (rc) return rc;
  }
  // fallback for flagged panels (rank deficient or with a structurally zero
  // column): every kernel is gated on the flag
  rc = panel_columns(cx, rowmajor, P, ldp, m, nb, V, ldv, tau, pw, counter, panel_rows, flag, 1, s);
  if (rc) return rc;
  rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, P_F64, nb, nb, m, V, ldv, V, ldv, pw.S, nb, 1.0, 0.0, s,
            flag, 1);
  if (rc) return rc;
  ProfScope p3(C_LARFT, 0.0, s);
  return launch_larft(pw.S, nb, tau, nb, T, ldt, s, flag, 1);
}

// ---------------------------------------------------------------------------
// SY2SB
// ---------------------------------------------------------------------------
// na: the no-allocation state (static scratch, one stream, no events), or
// nullptr for the library's own workspace.
static int sy2sb_impl(int64_t n64, int64_t w64, int64_t b64, double *A, int64_t lda, double *tau,
                      int prec, const bandred_opts_t *opts, hipStream_t s,
                      DevState *na = nullptr) {
  if (n64 <= w64 + 1) {
    if (n64 > w64) return launch_fill(tau, n64 - w64, 0.0, s);  // one trivial reflector
    return 0;
  }
  if (n64 > (int64_t)1 << 30) return BANDRED_ERR_UNSUPPORTED;
  const int n = (int)n64, w = (int)w64, b = (int)b64;
  const int lookahead = na ? 0 : (opts ? opts->lookahead : 1);
  const int panel_rows = opts ? opts->panel_rows : 0;
  const int method = opts ? opts->panel_method : 0;
  DevState *st = na;
  int rc = na ? 0 : dev_state(&st);
  if (rc) return rc;

  const int nref = n - w - 1;  // reflector columns 0 .. n-w-2
  const int npan = (nref + b - 1) / b;
  const int jmax = n - w;      // rows of the first panel
  const size_t part_main = std::max<size_t>((size_t)8 * jmax * b, (size_t)256 * b * b);
  const size_t part_pan = (size_t)(jmax / 64 + 2) * b * b;
  size_t need = 0;
  need += 2 * round_up((size_t)jmax * 2 * b * 8, 256);   // WV[2] = [W | V]
  need += 2 * round_up((size_t)jmax * b * 8, 256);       // Wt[2] = V T
  need += round_up(part_main * 8, 256) + round_up(part_pan * 8, 256);
  need += 4 * round_up((size_t)b * std::max(b, w) * 8, 256);  // T[2], M, Z
  need += PanelWs::bytes(jmax, b);
  need += 3 * round_up((size_t)(npan + 1) * 4, 256);     // counters, flags (2 per panel)
  need += round_up((size_t)(npan + 1) * 2 * kNbMax * 4, 256);  // panel structure
  const size_t oz_sz = prec == P_OZ ? oz_bound(jmax, jmax, 2 * std::max(b, w)) : 0;
  need += oz_sz;
  if (prec == P_OZ) need += round_up((size_t)jmax * 8, 256);  // row maxima of A2
  need += 8192;
  std::lock_guard<std::mutex> lk(g_mu);
  bool capturing = false;
  if (na) {
    if (need > na->bytes || g_prof) return BANDRED_ERR_UNSUPPORTED;
  } else {
    rc = capture_check(s, need, *st, &capturing);
    if (rc) return rc;
    rc = ws_reserve(*st, need);
    if (rc) return rc;
  }
  // calls through the library's workspace are ordered on it by the
  // completion event of the previous call (not under capture, where the
  // caller orders replays, and not on the no-allocation path)
  const bool ordered = !capturing && !na;
  Arena ar(st->base);
  double *WVbuf[2] = {ar.take<double>((size_t)jmax * 2 * b), ar.take<double>((size_t)jmax * 2 * b)};
  double *Wtb[2] = {ar.take<double>((size_t)jmax * b), ar.take<double>((size_t)jmax * b)};
  double *partm = ar.take<double>(part_main);
  double *partp = ar.take<double>(part_pan);
  const size_t sq = (size_t)b * std::max(b, w);
  double *Tb[2] = {ar.take<double>(sq), ar.take<double>(sq)};
  double *Mb = ar.take<double>(sq), *Zb = ar.take<double>(sq);
  PanelWs pw;
  pw.carve(ar, jmax, b);
  unsigned *counters = ar.take<unsigned>(npan + 1);
  int *pflags = ar.take<int>(2 * (npan + 1));
  int *pstruct = ar.take<int>((size_t)(npan + 1) * 2 * kNbMax);

  Ctx cxm{st, s, partm, part_main};
  if (opts) {
    cxm.max_chunks = opts->update_chunks;
    cxm.lds_cap = opts->update_lds_cap;
  }
  unsigned long long *oz_rm = nullptr;  // row maxima of the trailing matrix (exact split)
  bool rm_valid = false;                // oz_rm holds those of this iteration's A2
  if (oz_sz) {
    cxm.oz = ar.take<char>(oz_sz);
    cxm.oz_cap = oz_sz;
    oz_rm = ar.take<unsigned long long>(jmax);
  }
  hipStream_t ps = lookahead ? st->aux : s;  // panel stream
  Ctx cxp{st, ps, partp, part_pan};

  if (ordered) BR_HIP_CHECK(hipStreamWaitEvent(s, st->done, 0));
  rc = launch_fill_u32(counters, npan + 1, 0u, s); if (rc) return rc;
  rc = launch_fill_u32((unsigned *)pflags, 2 * (npan + 1), 0u, s); if (rc) return rc;
  rc = launch_fill_u32((unsigned *)pstruct, (int64_t)(npan + 1) * 2 * kNbMax, 0u, s);
  if (rc) return rc;
  rc = launch_fill_u32((unsigned *)st->flags, 2, 0u, s); if (rc) return rc;
  g_last_flags[current_dev_index()] = st->flags;
  rc = launch_fill(tau, n - w, 0.0, s); if (rc) return rc;

  // panel `it` (columns c .. c+pb-1) and its Wt = V T, on stream q
  // The trailing update that runs beside a look-ahead panel waits for the
  // panel's head, its sparsity check and first Gram product P^T P (point 1 of
  // panel_factor), so that this wide product runs on the whole chip; the rest
  // of the panel (latency-bound b x b kernels and narrower products) then runs
  // beside the update.  Without it a graph replay, which dispatches both
  // branches at once, stretched both.  Measured: Variant V1 (SY2SB n=16384,
  // w=256, b=128) 164.2 -> 151.2 ms (eager calls, where the host issues the
  // panel's launches before the SYMM's, 150.7 against 152.8); Variant V2
  // (n=16384, w=b=128, the rest of the SYR2K waiting) 160.4 -> 158.6 ms.
  const int head_at = lookahead ? 1 : 0;
  bool head_recorded = false;  // set by the last factor() call that recorded ev_h
  auto factor = [&](int it, Ctx &cx, hipStream_t q) -> int {
    const int c = it * b, pb = std::min(b, nref - c), r = c + w, j = n - r;
    double *V = WVbuf[it & 1] + (int64_t)pb * j;
    const bool h = head_at > 0 && q != s;
    head_recorded = false;
    int e = panel_factor(cx, false, A + r + (int64_t)c * lda, lda, j, pb, V, j, tau + c,
                         Tb[it & 1], pb, pw, counters + it, pflags + 2 * it,
                         pstruct + (size_t)it * 2 * kNbMax, method, panel_rows, q,
                         h ? st->ev_h : nullptr, head_at, &head_recorded);
    if (e) return e;
    return gemm(cx, C_GEMM_SMALL, A_N, B_N, P_F64, j, pb, pb, V, j, Tb[it & 1], pb, Wtb[it & 1], j,
                1.0, 0.0, q);
  };

  rc = factor(0, cxm, s);
  if (rc) return rc;

  for (int it = 0, c = 0; c < nref; ++it, c += b) {
    const int pb = std::min(b, nref - c);
    const int r = c + w, j = n - r;
    double *WV = WVbuf[it & 1];
    double *W = WV, *V = WV + (int64_t)pb * j;
    double *Wt = Wtb[it & 1];
    double *A2 = A + r + (int64_t)r * lda;

    const int cn = c + b;
    const bool has_next = cn < nref;
    const int pbn = has_next ? std::min(b, nref - cn) : 0;
    const int a2L = has_next ? std::max(0, cn + pbn - r) : 0;  // A2 columns of the next panel

    auto fork_next = [&]() -> int {
      if (!has_next) return 0;
      if (ps != s) {
        BR_HIP_CHECK(hipEventRecord(st->ev_a, s));
        BR_HIP_CHECK(hipStreamWaitEvent(ps, st->ev_a, 0));
      }
      return factor(it + 1, cxp, ps);
    };

    // (3) A1 = A[r:n, c+pb : r] -= V T^T (V^T A1) = V (Wt^T A1)   (eq. updateA1)
    // Variant V1 (the next panel lies inside A1, 2b <= w): A1 is split as in
    // eq. partitionV1 into A1^L, the next panel's columns, which is updated
    // before the next panel is forked, and A1^R, updated on the main stream
    // beside that panel together with A2.
    const int a1w = w - pb;
    auto update_a1 = [&](int q0, int q1) -> int {  // A1 columns [q0, q1)
      if (q1 <= q0) return 0;
      double *A1 = A + r + (int64_t)(c + pb + q0) * lda;
      int e = gemm(cxm, C_GEMM_SMALL, A_T, B_N, P_F64, pb, q1 - q0, j, Wt, j, A1, lda, Zb, pb,
                   1.0, 0.0, s);
      if (e) return e;
      return gemm(cxm, C_GEMM_UPD, A_N, B_N, prec, j, q1 - q0, pb, V, j, Zb, pb, A1, lda, -1.0,
                  1.0, s);
    };
    const bool v1 = has_next && a2L == 0;
    const int a1L = v1 ? std::min(a1w, cn + pbn - (c + pb)) : a1w;  // A1^L: A1 columns [0, a1L)
    rc = update_a1(0, a1L);
    if (rc) return rc;
    if (v1) {
      rc = fork_next();
      if (rc) return rc;
      if (head_recorded) BR_HIP_CHECK(hipStreamWaitEvent(s, st->ev_h, 0));
    }
    rc = update_a1(a1L, a1w);  // A1^R (empty in Variant V2)
    if (rc) return rc;
    // (4) X = A2 Wt (SYMM) into W's slot; M = Wt^T X; W = X - 1/2 V M
    if (rm_valid) cxm.oz_rmax_in = oz_rm;
    rc = gemm(cxm, C_SYMM, A_SYM, B_N, prec, j, pb, j, A2, lda, Wt, j, W, j, 1.0, 0.0, s);
    cxm.oz_rmax_in = nullptr;
    if (rc) return rc;
    rc = gemm(cxm, C_GEMM_SMALL, A_T, B_N, P_F64, pb, pb, j, Wt, j, W, j, Mb, pb, 1.0, 0.0, s);
    if (rc) return rc;
    rc = gemm(cxm, C_GEMM_SMALL, A_N, B_N, P_F64, j, pb, pb, V, j, Mb, pb, W, j, -0.5, 1.0, s);
    if (rc) return rc;
    // (6) SYR2K: the next panel's columns A2^L first, then fork (Variant V2)
    rc = syr2k(cxm, prec, j, pb, WV, j, A2, lda, 0, a2L, s);
    if (rc) return rc;
    if (a2L > 0) {
      rc = fork_next();
      if (rc) return rc;
      if (head_recorded) BR_HIP_CHECK(hipStreamWaitEvent(s, st->ev_h, 0));
    }
    // the rest beside the next panel: in chunks (see update_chunks).  In the
    // exact split it writes every stored entry of the next trailing matrix
    // (columns >= b, the next panel's columns lying below b) and records its
    // row maxima for the next SYMM.
    rm_valid = false;
    if (prec == P_OZ && has_next) {
      rc = launch_fill_u32((unsigned *)oz_rm, 2 * (int64_t)(j - b), 0u, s);
      if (rc) return rc;
      cxm.oz_rec = oz_rm;
      cxm.oz_rec_off = b;
      rm_valid = true;
    }
    if (has_next && ps != s)
      rc = syr2k_chunked(cxm, prec, j, pb, WV, j, A2, lda, a2L, j, s);
    else
      rc = syr2k(cxm, prec, j, pb, WV, j, A2, lda, a2L, j, s);
    cxm.oz_rec = nullptr;
    cxm.oz_rec_off = 0;
    if (rc) return rc;
    if (has_next && ps != s) {
      BR_HIP_CHECK(hipEventRecord(st->ev_b, ps));
      BR_HIP_CHECK(hipStreamWaitEvent(s, st->ev_b, 0));
    }
  }
  if (ordered) BR_HIP_CHECK(hipEventRecord(st->done, s));
  return 0;
}

// ---------------------------------------------------------------------------
// GE2GB
// ---------------------------------------------------------------------------
static int ge2gb_impl(int64_t m64, int64_t n64, int64_t w64, int64_t b64, double *A, int64_t lda,
                      double *tauq, double *taup, int prec, const bandred_opts_t *opts,
                      hipStream_t s) {
  if (n64 == 0) return 0;
  if (m64 > (int64_t)1 << 30) return BANDRED_ERR_UNSUPPORTED;
  const int m = (int)m64, n = (int)n64, w = (int)w64, b = (int)b64;
  const int panel_rows = opts ? opts->panel_rows : 0;
  const int method = opts ? opts->panel_method : 0;
  // look-ahead when the next left panel is the first column block of D (w = b)
  const bool la = (opts ? opts->lookahead : 1) && w == b;
  DevState *st = nullptr;
  int rc = dev_state(&st);
  if (rc) return rc;
  const int npan = (n + b - 1) / b;
  const size_t part_cap = std::max<size_t>((size_t)8 * m * b, (size_t)256 * b * b);
  const size_t part_pan = (size_t)(m / 64 + 2) * b * b;
  size_t need = 0;
  need += 2 * round_up((size_t)m * b * 8, 256);       // Vq, Wtq
  need += 2 * round_up((size_t)n * b * 8, 256);       // Up, Wtp
  need += round_up((size_t)b * n * 8, 256);           // Z (b x n)
  need += round_up((size_t)m * b * 8, 256);           // X (m x b)
  need += round_up(part_cap * 8, 256) + round_up(part_pan * 8, 256);
  need += 2 * round_up((size_t)b * b * 8, 256);       // Tq, Tp
  need += PanelWs::bytes(m, b);
  need += 3 * round_up((size_t)(2 * npan + 2) * 4, 256);
  need += round_up((size_t)(2 * npan + 2) * 2 * kNbMax * 4, 256);  // panel structure
  const size_t oz_sz = prec == P_OZ ? oz_bound(m, n, 2 * std::max(b, w)) : 0;
  need += oz_sz;
  need += 8192;
  std::lock_guard<std::mutex> lk(g_mu);
  bool capturing = false;
  rc = capture_check(s, need, *st, &capturing);
  if (rc) return rc;
  rc = ws_reserve(*st, need);
  if (rc) return rc;
  Arena ar(st->base);
  double *Vq = ar.take<double>((size_t)m * b), *Wtq = ar.take<double>((size_t)m * b);
  double *Up = ar.take<double>((size_t)n * b), *Wtp = ar.take<double>((size_t)n * b);
  double *Zb = ar.take<double>((size_t)b * n);
  double *Xb = ar.take<double>((size_t)m * b);
  double *part = ar.take<double>(part_cap);
  double *partp = ar.take<double>(part_pan);
  double *Tq = ar.take<double>((size_t)b * b), *Tp = ar.take<double>((size_t)b * b);
  PanelWs pw;
  pw.carve(ar, m, b);
  unsigned *counters = ar.take<unsigned>(2 * npan + 2);
  int *pflags = ar.take<int>(2 * (2 * npan + 2));
  int *pstruct = ar.take<int>((size_t)(2 * npan + 2) * 2 * kNbMax);
  Ctx cx{st, s, part, part_cap};
  if (opts) {
    cx.max_chunks = opts->update_chunks;
    cx.lds_cap = opts->update_lds_cap;
  }
  if (oz_sz) {
    cx.oz = ar.take<char>(oz_sz);
    cx.oz_cap = oz_sz;
  }
  hipStream_t ps = la ? st->aux : s;  // panel stream
  Ctx cxp{st, ps, partp, part_pan};  // panels: their own split-k buffer on either stream

  if (!capturing) BR_HIP_CHECK(hipStreamWaitEvent(s, st->done, 0));
  rc = launch_fill_u32(counters, 2 * npan + 2, 0u, s); if (rc) return rc;
  rc = launch_fill_u32((unsigned *)pflags, 2 * (2 * npan + 2), 0u, s); if (rc) return rc;
  rc = launch_fill_u32((unsigned *)pstruct, (int64_t)(2 * npan + 2) * 2 * kNbMax, 0u, s);
  if (rc) return rc;
  rc = launch_fill_u32((unsigned *)st->flags, 2, 0u, s); if (rc) return rc;
  g_last_flags[current_dev_index()] = st->flags;
  rc = launch_fill(tauq, n, 0.0, s); if (rc) return rc;
  rc = launch_fill(taup, n, 0.0, s); if (rc) return rc;

  // left panel `it` (columns c .. c+pb-1) and Wtq = Vq Tq, on stream q
  // a panel forked beside an update records the head event (see sy2sb_impl)
  bool head_recorded = false;
  auto left_panel = [&](int it, Ctx &c_, hipStream_t q) -> int {
    const int c = it * b, pb = std::min(b, n - c), i = m - c;
    head_recorded = false;
    int r = panel_factor(c_, false, A + c + (int64_t)c * lda, lda, i, pb, Vq, i, tauq + c, Tq, pb,
                         pw, counters + 2 * it, pflags + 4 * it,
                         pstruct + (size_t)(2 * it) * 2 * kNbMax, method, panel_rows, q,
                         q != s ? st->ev_h : nullptr, 1, &head_recorded);
    if (r) return r;
    return gemm(c_, C_GEMM_SMALL, A_N, B_N, P_F64, i, pb, pb, Vq, i, Tq, pb, Wtq, i, 1.0, 0.0, q);
  };
  // right panel of step `it` (rows c .. c+pr-1 from column c+w) and Wtp = Up Tp
  auto right_panel = [&](int it, Ctx &c_, hipStream_t q) -> int {
    const int c = it * b, pb = std::min(b, n - c);
    const int pr = std::max(0, std::min(pb, n - w - 1 - c));
    const int c0 = c + w, jr = n - c0;
    head_recorded = false;
    int r = panel_factor(c_, true, A + c + (int64_t)c0 * lda, lda, jr, pr, Up, jr, taup + c, Tp, pr,
                         pw, counters + 2 * it + 1, pflags + 4 * it + 2,
                         pstruct + (size_t)(2 * it + 1) * 2 * kNbMax, method, panel_rows, q,
                         q != s ? st->ev_h : nullptr, 1, &head_recorded);
    if (r) return r;
    return gemm(c_, C_GEMM_SMALL, A_N, B_N, P_F64, jr, pr, pr, Up, jr, Tp, pr, Wtp, jr, 1.0, 0.0, q);
  };

  // Per step (Sec. 3.1): (1) left QR, Wtq = Vq Tq; (2) E -= Vq (Wtq^T E);
  // (3) right LQ of the updated top rows, Wtp = Up Tp; (4) D -= (D Wtp) Up^T.
  // With look-ahead the panels run on the panel stream: (3) as soon as the
  // top rows of E are updated (overlapping the rest of (2)), and the next
  // step's (1) as soon as the first column block of D is updated
  // (overlapping the rest of (4)).
  if (la) {
    BR_HIP_CHECK(hipEventRecord(st->ev_a, s));
    BR_HIP_CHECK(hipStreamWaitEvent(ps, st->ev_a, 0));
  }
  rc = left_panel(0, cxp, ps);
  if (rc) return rc;
  if (la) {
    BR_HIP_CHECK(hipEventRecord(st->ev_b, ps));
    BR_HIP_CHECK(hipStreamWaitEvent(s, st->ev_b, 0));
  }
  for (int it = 0, c = 0; c < n; ++it, c += b) {
    const int pb = std::min(b, n - c);
    const int i = m - c;
    const int pr = std::max(0, std::min(pb, n - w - 1 - c));
    const int ne = n - c - pb;
    // (2) E = A[c:m, c+pb:n] -= Vq (Wtq^T E): top pr rows first
    if (ne > 0) {
      double *E = A + c + (int64_t)(c + pb) * lda;
      rc = gemm(cx, C_GEMM_UPD, A_T, B_N, prec, pb, ne, i, Wtq, i, E, lda, Zb, pb, 1.0, 0.0, s);
      if (rc) return rc;
      const int top = (la && pr > 0) ? pr : i;
      rc = gemm(cx, C_GEMM_UPD, A_N, B_N, prec, top, ne, pb, Vq, i, Zb, pb, E, lda, -1.0, 1.0, s);
      if (rc) return rc;
      if (top < i) {
        BR_HIP_CHECK(hipEventRecord(st->ev_c, s));
        BR_HIP_CHECK(hipStreamWaitEvent(ps, st->ev_c, 0));
        rc = right_panel(it, cxp, ps);  // (3) overlaps the rest of (2)
        if (rc) return rc;
        if (head_recorded) BR_HIP_CHECK(hipStreamWaitEvent(s, st->ev_h, 0));
        BR_HIP_CHECK(hipEventRecord(st->ev_d, ps));
        rc = gemm_chunked(cx, C_GEMM_UPD, A_N, B_N, prec, i - top, ne, pb, Vq + top, i, Zb, pb,
                          E + top, lda, -1.0, 1.0, s);
        if (rc) return rc;
        BR_HIP_CHECK(hipStreamWaitEvent(s, st->ev_d, 0));
      } else if (pr > 0) {
        rc = right_panel(it, cxp, s);
        if (rc) return rc;
      }
    } else if (pr > 0) {
      rc = right_panel(it, cxp, s);
      if (rc) return rc;
    }
    const bool next = (c + pb < n);
    if (pr > 0) {
      // (4) D = A[c+pr:m, c0:n] -= (D Wtp) Up^T
      const int c0 = c + w, jr = n - c0;
      const int md = m - c - pr;
      if (md > 0) {
        double *D = A + (c + pr) + (int64_t)c0 * lda;
        rc = gemm(cx, C_GEMM_UPD, A_N, B_N, prec, md, pr, jr, D, lda, Wtp, jr, Xb, md, 1.0, 0.0, s);
        if (rc) return rc;
        // with w = b and pr = pb the next left panel is D's first column block
        const int lcols = (la && next && pr == pb) ? std::min(b, jr) : 0;
        if (lcols > 0) {
          rc = gemm(cx, C_GEMM_UPD, A_N, B_T, prec, md, lcols, pr, Xb, md, Up, jr, D, lda, -1.0,
                    1.0, s);
          if (rc) return rc;
          BR_HIP_CHECK(hipEventRecord(st->ev_a, s));
          BR_HIP_CHECK(hipStreamWaitEvent(ps, st->ev_a, 0));
          rc = left_panel(it + 1, cxp, ps);  // next (1) overlaps the rest of (4)
          if (rc) return rc;
          if (head_recorded) BR_HIP_CHECK(hipStreamWaitEvent(s, st->ev_h, 0));
          BR_HIP_CHECK(hipEventRecord(st->ev_b, ps));
          if (jr > lcols) {
            rc = gemm_chunked(cx, C_GEMM_UPD, A_N, B_T, prec, md, jr - lcols, pr, Xb, md,
                              Up + lcols, jr, D + (int64_t)lcols * lda, lda, -1.0, 1.0, s);
            if (rc) return rc;
          }
          BR_HIP_CHECK(hipStreamWaitEvent(s, st->ev_b, 0));
          continue;
        }
        rc = gemm(cx, C_GEMM_UPD, A_N, B_T, prec, md, jr, pr, Xb, md, Up, jr, D, lda, -1.0, 1.0, s);
        if (rc) return rc;
      }
    }
    if (next) {
      if (la) {
        BR_HIP_CHECK(hipEventRecord(st->ev_a, s));
        BR_HIP_CHECK(hipStreamWaitEvent(ps, st->ev_a, 0));
      }
      rc = left_panel(it + 1, cxp, ps);
      if (rc) return rc;
      if (la) {
        BR_HIP_CHECK(hipEventRecord(st->ev_b, ps));
        BR_HIP_CHECK(hipStreamWaitEvent(s, st->ev_b, 0));
      }
    }
  }
  if (!capturing) BR_HIP_CHECK(hipEventRecord(st->done, s));
  return 0;
}

// ---------------------------------------------------------------------------
// GE2GB to the band form with equal lower and upper bandwidth (Sec. 3.3).
// Per block c (left panel width pbl, right panel width pbr):
//   1. left QR of B0 = A[c+w:m, c:c+pbl], Wtl = Vl Tl           (eq. updateB0)
//      right LQ of C0 = A[c:c+pbr, c+w:n], Wtr = Vr Tr          (eq. updateC0)
//      (independent: their reflectors touch disjoint rows and columns)
//   2. B1 = A[c+w:m, c+pbl:c+w] -= Vl (Wtl^T B1)                  (eq. updateBD)
//      C1 = A[c+pbr:c+w, c+w:n] -= (C1 Wtr) Vr^T                  (eq. updateCD2)
//   3. D = A[c+w:m, c+w:n], both sides at once (eq. gebrd_2k):
//      ZL = D^T Wtl, ZR = D Wtr, X = ZR - Vl (ZL^T Wtr),
//      D -= [X, Vl] [Vr, ZL]^T
// The paper's Q_L = I + W_L Y_L^T is I - Vl Tl Vl^T here (Y = V, W = -V T),
// so its X and Z_L carry the opposite sign.
// Look-ahead: when the next panels lie in B1 and C1 (Variant V1, 2b <= w)
// they are factored on the second stream right after step 2, beside the whole
// of step 3; otherwise (Variant V2) the parts of D that the next panels need
// (D11, D21 and D12 of eq. partD) are updated first and the rest (D22)
// beside the next panels.
// ---------------------------------------------------------------------------
static int ge2gb_lu_impl(int64_t m64, int64_t n64, int64_t w64, int64_t b64, double *A,
                         int64_t lda, double *tauq, double *taup, int prec,
                         const bandred_opts_t *opts, hipStream_t s) {
  if (n64 == 0) return 0;
  if (m64 > (int64_t)1 << 30) return BANDRED_ERR_UNSUPPORTED;
  const int m = (int)m64, n = (int)n64, w = (int)w64, b = (int)b64;
  const int panel_rows = opts ? opts->panel_rows : 0;
  const int method = opts ? opts->panel_method : 0;
  const bool la = opts ? opts->lookahead != 0 : true;
  DevState *st = nullptr;
  int rc = dev_state(&st);
  if (rc) return rc;
  // reflectors of length >= 2: left c <= m-w-2, right c <= n-w-2
  const int nl = std::max(0, std::min(n, m - w - 1));
  const int nr = std::max(0, n - w - 1);
  const int npan = (nl + b - 1) / b;
  if (npan == 0) {  // already banded: every tau is zero
    rc = launch_fill(tauq, n, 0.0, s); if (rc) return rc;
    return launch_fill(taup, n, 0.0, s);
  }
  const int jlmax = m - w, jrmax = std::max(1, n - w);
  const size_t part_cap = std::max<size_t>((size_t)8 * std::max(jlmax, jrmax) * b,
                                           (size_t)256 * b * b);
  const size_t part_pan = (size_t)(std::max(jlmax, jrmax) / 64 + 2) * b * b;
  size_t need = 0;
  need += 2 * round_up((size_t)jlmax * 2 * b * 8, 256);  // XV[2] = [X | Vl]
  need += 2 * round_up((size_t)jrmax * 2 * b * 8, 256);  // VZ[2] = [Vr | ZL]
  need += 2 * round_up((size_t)jlmax * b * 8, 256);      // Wtl[2]
  need += 2 * round_up((size_t)jrmax * b * 8, 256);      // Wtr[2]
  need += 4 * round_up((size_t)b * b * 8, 256);          // Tl[2], Tr[2]
  need += 3 * round_up((size_t)b * std::max(b, w) * 8, 256);  // Zb, Yc, P
  need += round_up(part_cap * 8, 256) + round_up(part_pan * 8, 256);
  need += PanelWs::bytes(std::max(jlmax, jrmax), b);
  need += 3 * round_up((size_t)(2 * npan + 2) * 4, 256);
  need += round_up((size_t)(2 * npan + 2) * 2 * kNbMax * 4, 256);
  const size_t oz_sz = prec == P_OZ ? oz_bound(m, n, 2 * std::max(b, w)) : 0;
  need += oz_sz;
  need += 8192;
  std::lock_guard<std::mutex> lk(g_mu);
  bool capturing = false;
  rc = capture_check(s, need, *st, &capturing);
  if (rc) return rc;
  rc = ws_reserve(*st, need);
  if (rc) return rc;
  Arena ar(st->base);
  double *XV[2] = {ar.take<double>((size_t)jlmax * 2 * b), ar.take<double>((size_t)jlmax * 2 * b)};
  double *VZ[2] = {ar.take<double>((size_t)jrmax * 2 * b), ar.take<double>((size_t)jrmax * 2 * b)};
  double *Wtl[2] = {ar.take<double>((size_t)jlmax * b), ar.take<double>((size_t)jlmax * b)};
  double *Wtr[2] = {ar.take<double>((size_t)jrmax * b), ar.take<double>((size_t)jrmax * b)};
  double *Tl[2] = {ar.take<double>((size_t)b * b), ar.take<double>((size_t)b * b)};
  double *Tr[2] = {ar.take<double>((size_t)b * b), ar.take<double>((size_t)b * b)};
  const size_t sq = (size_t)b * std::max(b, w);
  double *Zb = ar.take<double>(sq), *Yc = ar.take<double>(sq), *Pb = ar.take<double>(sq);
  double *part = ar.take<double>(part_cap);
  double *partp = ar.take<double>(part_pan);
  PanelWs pw;
  pw.carve(ar, std::max(jlmax, jrmax), b);
  unsigned *counters = ar.take<unsigned>(2 * npan + 2);
  int *pflags = ar.take<int>(2 * (2 * npan + 2));
  int *pstruct = ar.take<int>((size_t)(2 * npan + 2) * 2 * kNbMax);
  Ctx cx{st, s, part, part_cap};
  if (opts) {
    cx.max_chunks = opts->update_chunks;
    cx.lds_cap = opts->update_lds_cap;
  }
  if (oz_sz) {
    cx.oz = ar.take<char>(oz_sz);
    cx.oz_cap = oz_sz;
  }
  hipStream_t ps = la ? st->aux : s;
  Ctx cxp{st, ps, partp, part_pan};

  if (!capturing) BR_HIP_CHECK(hipStreamWaitEvent(s, st->done, 0));
  rc = launch_fill_u32(counters, 2 * npan + 2, 0u, s); if (rc) return rc;
  rc = launch_fill_u32((unsigned *)pflags, 2 * (2 * npan + 2), 0u, s); if (rc) return rc;
  rc = launch_fill_u32((unsigned *)pstruct, (int64_t)(2 * npan + 2) * 2 * kNbMax, 0u, s);
  if (rc) return rc;
  rc = launch_fill_u32((unsigned *)st->flags, 2, 0u, s); if (rc) return rc;
  g_last_flags[current_dev_index()] = st->flags;
  rc = launch_fill(tauq, n, 0.0, s); if (rc) return rc;
  rc = launch_fill(taup, n, 0.0, s); if (rc) return rc;

  bool head_recorded = false;  // the left panel forked last recorded ev_h (see sy2sb_impl)
  auto widths = [&](int c, int *pbl, int *pbr) {
    *pbl = std::max(0, std::min(b, nl - c));
    *pbr = std::max(0, std::min(b, nr - c));
  };
  // both panels of block `it` and their Wt = V T, on stream q
  auto panels = [&](int it, Ctx &c_, hipStream_t q) -> int {
    const int c = it * b, jl = m - c - w, jr = n - c - w;
    int pbl, pbr;
    widths(c, &pbl, &pbr);
    const int k = it & 1;
    if (pbl > 0) {
      double *Vl = XV[k] + (int64_t)pbr * jl;  // [X | Vl]: Vl after the pbr columns of X
      int r = panel_factor(c_, false, A + (c + w) + (int64_t)c * lda, lda, jl, pbl, Vl, jl,
                           tauq + c, Tl[k], pbl, pw, counters + 2 * it, pflags + 4 * it,
                           pstruct + (size_t)(2 * it) * 2 * kNbMax, method, panel_rows, q,
                           q != s ? st->ev_h : nullptr, 1, &head_recorded);
      if (r) return r;
      r = gemm(c_, C_GEMM_SMALL, A_N, B_N, P_F64, jl, pbl, pbl, Vl, jl, Tl[k], pbl, Wtl[k], jl,
               1.0, 0.0, q);
      if (r) return r;
    }
    if (pbr > 0) {
      double *Vr = VZ[k];  // [Vr | ZL]
      int r = panel_factor(c_, true, A + c + (int64_t)(c + w) * lda, lda, jr, pbr, Vr, jr,
                           taup + c, Tr[k], pbr, pw, counters + 2 * it + 1, pflags + 4 * it + 2,
                           pstruct + (size_t)(2 * it + 1) * 2 * kNbMax, method, panel_rows, q);
      if (r) return r;
      r = gemm(c_, C_GEMM_SMALL, A_N, B_N, P_F64, jr, pbr, pbr, Vr, jr, Tr[k], pbr, Wtr[k], jr,
               1.0, 0.0, q);
      if (r) return r;
    }
    return 0;
  };
  auto fork = [&](int it) -> int {
    if (ps != s) {
      BR_HIP_CHECK(hipEventRecord(st->ev_a, s));
      BR_HIP_CHECK(hipStreamWaitEvent(ps, st->ev_a, 0));
    }
    head_recorded = false;
    int r = panels(it, cxp, ps);
    if (r) return r;
    if (head_recorded) BR_HIP_CHECK(hipStreamWaitEvent(s, st->ev_h, 0));
    return 0;
  };
  auto join = [&]() -> int {
    if (ps != s) {
      BR_HIP_CHECK(hipEventRecord(st->ev_b, ps));
      BR_HIP_CHECK(hipStreamWaitEvent(s, st->ev_b, 0));
    }
    return 0;
  };

  rc = panels(0, cx, s);
  if (rc) return rc;
  for (int it = 0; it < npan; ++it) {
    const int c = it * b, jl = m - c - w, jr = n - c - w;
    int pbl, pbr;
    widths(c, &pbl, &pbr);
    const int k = it & 1;
    double *Vl = XV[k] + (int64_t)pbr * jl, *Vr = VZ[k];
    const bool next = it + 1 < npan;
    int pbl2 = 0, pbr2 = 0;
    if (next) widths(c + b, &pbl2, &pbr2);
    // columns / rows of D that the next panels take (Variant V2 when nonzero)
    const int aL = next ? std::max(0, std::min(jr, c + b + pbl2 - (c + w))) : 0;
    const int aR = next ? std::max(0, std::min(jl, c + b + pbr2 - (c + w))) : 0;

    // (2) B1 and C1
    const int nb1 = std::min(c + w, n) - (c + pbl);
    if (pbl > 0 && nb1 > 0) {
      double *B1 = A + (c + w) + (int64_t)(c + pbl) * lda;
      rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, prec, pbl, nb1, jl, Wtl[k], jl, B1, lda, Zb, pbl,
                1.0, 0.0, s);
      if (rc) return rc;
      rc = gemm(cx, C_GEMM_UPD, A_N, B_N, prec, jl, nb1, pbl, Vl, jl, Zb, pbl, B1, lda, -1.0,
                1.0, s);
      if (rc) return rc;
    }
    const int mc1 = std::min(c + w, m) - (c + pbr);
    if (pbr > 0 && mc1 > 0) {
      double *C1 = A + (c + pbr) + (int64_t)(c + w) * lda;
      rc = gemm(cx, C_GEMM_SMALL, A_N, B_N, prec, mc1, pbr, jr, C1, lda, Wtr[k], jr, Yc, mc1,
                1.0, 0.0, s);
      if (rc) return rc;
      rc = gemm(cx, C_GEMM_UPD, A_N, B_T, prec, mc1, jr, pbr, Yc, mc1, Vr, jr, C1, lda, -1.0,
                1.0, s);
      if (rc) return rc;
    }
    const bool v1 = next && aL == 0 && aR == 0;
    if (v1) {
      rc = fork(it + 1);
      if (rc) return rc;
    }
    // (3) D, both sides at once
    if (jr > 0 && jl > 0) {
      double *D = A + (c + w) + (int64_t)(c + w) * lda;
      double *ZL = VZ[k] + (int64_t)pbr * jr;
      double *X = XV[k];
      if (pbl > 0) {  // ZL = D^T Wtl
        rc = gemm(cx, C_GEMM_UPD, A_T, B_N, prec, jr, pbl, jl, D, lda, Wtl[k], jl, ZL, jr, 1.0,
                  0.0, s);
        if (rc) return rc;
      }
      if (pbr > 0) {  // ZR = D Wtr into X's slot; X = ZR - Vl (ZL^T Wtr)
        rc = gemm(cx, C_GEMM_UPD, A_N, B_N, prec, jl, pbr, jr, D, lda, Wtr[k], jr, X, jl, 1.0,
                  0.0, s);
        if (rc) return rc;
        if (pbl > 0) {
          rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, P_F64, pbl, pbr, jr, ZL, jr, Wtr[k], jr, Pb, pbl,
                    1.0, 0.0, s);
          if (rc) return rc;
          rc = gemm(cx, C_GEMM_SMALL, A_N, B_N, P_F64, jl, pbr, pbl, Vl, jl, Pb, pbl, X, jl,
                    -1.0, 1.0, s);
          if (rc) return rc;
        }
      }
      // D -= [X | Vl] [Vr | ZL]^T over the rank pbr + pbl
      const int K = pbr + pbl;
      auto upd = [&](int r0, int r1, int c0, int c1, bool chunked) -> int {
        if (r1 <= r0 || c1 <= c0) return 0;
        // (the exact-split form scales X and Vl apart: see gemm_oz)
        if (chunked)
          return gemm_chunked(cx, C_GEMM_UPD, A_N, B_T, prec, r1 - r0, c1 - c0, K, X + r0, jl,
                              VZ[k] + c0, jr, D + r0 + (int64_t)c0 * lda, lda, -1.0, 1.0, s, pbr);
        return gemm(cx, C_GEMM_UPD, A_N, B_T, prec, r1 - r0, c1 - c0, K, X + r0, jl, VZ[k] + c0,
                    jr, D + r0 + (int64_t)c0 * lda, lda, -1.0, 1.0, s, nullptr, 0, nullptr, 0, 0,
                    0, pbr);
      };
      if (next && !v1 && ps != s) {
        rc = upd(0, jl, 0, aL, false);   // D11 and D21: the next left panel's columns
        if (rc) return rc;
        rc = upd(0, aR, aL, jr, false);  // D12: the next right panel's rows
        if (rc) return rc;
        rc = fork(it + 1);
        if (rc) return rc;
        rc = upd(aR, jl, aL, jr, true);  // D22 beside the next panels
        if (rc) return rc;
      } else {
        rc = upd(0, jl, 0, jr, v1 && ps != s);
        if (rc) return rc;
      }
    }
    if (next) {
      if (v1 || (jr > 0 && jl > 0 && ps != s)) {
        rc = join();
      } else {
        rc = panels(it + 1, cx, s);  // serial order (or no D left to overlap)
      }
      if (rc) return rc;
    }
  }
  if (!capturing) BR_HIP_CHECK(hipEventRecord(st->done, s));
  return 0;
}

// ---------------------------------------------------------------------------
// Back-transformation: C := Q C or Q^T C for the stored reflectors of a
// reduction, Q = H_0 H_1 ... H_{nrefl-1} with reflector i acting on indices
// i+off .. len-1 (its vector in column i, or row i for right reflectors).
// Blocks of b reflectors are applied as I - V T V^T (Q^T: I - V T^T V^T),
// the compact WY form in which the reductions accumulate Q (Sec. 2.1,
// Q = I + W Y^T): V copied out of the storage, T from V^T V and tau (the
// LARFT recurrence), then C -= V (op(T) (V^T C)).
// ---------------------------------------------------------------------------
static int apply_impl(int rowstore, int64_t off, int64_t nrefl, int64_t len, const double *A,
                      int64_t lda, const double *tau, int trans, int64_t k64, double *C,
                      int64_t ldc, int b, hipStream_t s) {
  if (nrefl <= 0 || k64 <= 0) return 0;
  if (len > ((int64_t)1 << 30) || k64 > ((int64_t)1 << 30)) return BANDRED_ERR_UNSUPPORTED;
  const int k = (int)k64;
  DevState *st = nullptr;
  int rc = dev_state(&st);
  if (rc) return rc;
  const int jmax = (int)(len - off);
  const size_t part_cap = std::max<size_t>((size_t)8 * b * std::max(k, b), (size_t)256 * b * b);
  size_t need = round_up((size_t)jmax * b * 8, 256) + 2 * round_up((size_t)b * b * 8, 256) +
                2 * round_up((size_t)b * k * 8, 256) + round_up(part_cap * 8, 256) + 4096;
  std::lock_guard<std::mutex> lk(g_mu);
  bool capturing = false;
  rc = capture_check(s, need, *st, &capturing);
  if (rc) return rc;
  rc = ws_reserve(*st, need);
  if (rc) return rc;
  Arena ar(st->base);
  double *V = ar.take<double>((size_t)jmax * b);
  double *S = ar.take<double>((size_t)b * b), *T = ar.take<double>((size_t)b * b);
  double *Z = ar.take<double>((size_t)b * k), *Z2 = ar.take<double>((size_t)b * k);
  double *part = ar.take<double>(part_cap);
  Ctx cx{st, s, part, part_cap};
  if (!capturing) BR_HIP_CHECK(hipStreamWaitEvent(s, st->done, 0));
  rc = launch_fill_u32((unsigned *)st->flags, 2, 0u, s); if (rc) return rc;
  g_last_flags[current_dev_index()] = st->flags;
  const int nblk = (int)((nrefl + b - 1) / b);
  for (int q = 0; q < nblk; ++q) {
    const int bi = trans ? q : nblk - 1 - q;  // Q C: last block first
    const int64_t i0 = (int64_t)bi * b;
    const int pb = (int)std::min<int64_t>(b, nrefl - i0);
    const int64_t r0 = i0 + off;
    const int j = (int)(len - r0);
    double *Cr = C + r0;
    rc = launch_extract_v(A, lda, rowstore, r0, i0, pb, j, V, j, s);
    if (rc) return rc;
    rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, P_F64, pb, pb, j, V, j, V, j, S, pb, 1.0, 0.0, s);
    if (rc) return rc;
    {
      ProfScope p2(C_LARFT, 0.0, s);
      rc = launch_larft(S, pb, tau + i0, pb, T, pb, s);
      if (rc) return rc;
    }
    rc = gemm(cx, C_GEMM_UPD, A_T, B_N, P_F64, pb, k, j, V, j, Cr, ldc, Z, pb, 1.0, 0.0, s);
    if (rc) return rc;
    rc = gemm(cx, C_GEMM_SMALL, trans ? A_T : A_N, B_N, P_F64, pb, k, pb, T, pb, Z, pb, Z2, pb,
              1.0, 0.0, s);
    if (rc) return rc;
    rc = gemm(cx, C_GEMM_UPD, A_N, B_N, P_F64, j, k, pb, V, j, Z2, pb, Cr, ldc, -1.0, 1.0, s);
    if (rc) return rc;
  }
  if (!capturing) BR_HIP_CHECK(hipEventRecord(st->done, s));
  return 0;
}

// ---------------------------------------------------------------------------
// Stage 2 of the eigenvalue pipeline: the band left by SY2SB to tridiagonal
// form (bulge chasing, stage2.hip), and the tridiagonal matrix's eigenvalues.
// ---------------------------------------------------------------------------
static int sb2st_impl(int64_t n64, int64_t w64, const double *A, int64_t lda, double *dg,
                      double *e, hipStream_t s) {
  if (n64 == 0) return 0;
  if (n64 > ((int64_t)1 << 30)) return BANDRED_ERR_UNSUPPORTED;
  const int n = (int)n64;
  const int w = (int)std::min<int64_t>(w64, std::max<int64_t>(n64 - 1, 1));
  DevState *st = nullptr;
  int rc = dev_state(&st);
  if (rc) return rc;
  const int64_t ldab = 2 * (int64_t)w + 1;
  const size_t need = round_up((size_t)ldab * n * 8, 256) + round_up((size_t)n * 4, 256) + 1024;
  std::lock_guard<std::mutex> lk(g_mu);
  bool capturing = false;
  rc = capture_check(s, need, *st, &capturing);
  if (rc) return rc;
  rc = ws_reserve(*st, need);
  if (rc) return rc;
  Arena ar(st->base);
  double *AB = ar.take<double>((size_t)ldab * n);
  int *progress = ar.take<int>(n);
  unsigned *ctr = ar.take<unsigned>(64);
  if (!capturing) BR_HIP_CHECK(hipStreamWaitEvent(s, st->done, 0));
  rc = launch_fill_u32((unsigned *)progress, n, 0u, s); if (rc) return rc;
  rc = launch_fill_u32(ctr, 1, 0u, s); if (rc) return rc;
  rc = launch_fill_u32((unsigned *)st->flags, 2, 0u, s); if (rc) return rc;
  g_last_flags[current_dev_index()] = st->flags;
  rc = launch_sb2st(A, lda, n, w, AB, ldab, ctr, progress, st->flags, st->timeout_ticks,
                    st->num_cu, dg, e, s);
  if (rc) return rc;
  if (!capturing) BR_HIP_CHECK(hipEventRecord(st->done, s));
  return 0;
}

static int tridiag_eig_impl(int64_t n64, const double *dg, const double *e, double *lam,
                            hipStream_t s) {
  if (n64 == 0) return 0;
  if (n64 > ((int64_t)1 << 30)) return BANDRED_ERR_UNSUPPORTED;
  DevState *st = nullptr;
  int rc = dev_state(&st);
  if (rc) return rc;
  const size_t need = 1024;
  std::lock_guard<std::mutex> lk(g_mu);
  bool capturing = false;
  rc = capture_check(s, need, *st, &capturing);
  if (rc) return rc;
  rc = ws_reserve(*st, need);
  if (rc) return rc;
  Arena ar(st->base);
  double *bounds = ar.take<double>(8);
  if (!capturing) BR_HIP_CHECK(hipStreamWaitEvent(s, st->done, 0));
  rc = launch_fill_u32((unsigned *)st->flags, 2, 0u, s); if (rc) return rc;
  g_last_flags[current_dev_index()] = st->flags;
  rc = launch_tridiag_eig(dg, e, (int)n64, bounds, lam, s);
  if (rc) return rc;
  if (!capturing) BR_HIP_CHECK(hipEventRecord(st->done, s));
  return 0;
}

// ---------------------------------------------------------------------------
// Batched SY2SB: one persistent launch over a table of matrices sorted by
// decreasing order; matrices the kernel cannot hold (b > 16 or n - w > 1024)
// go through the single-matrix path on the same stream afterwards.
// ---------------------------------------------------------------------------
static int batched_impl(int64_t count, const int64_t *n, int w, int b, double *const *A,
                        const int64_t *lda, double *const *tau, int prec, hipStream_t s) {
  DevState *st = nullptr;
  int rc = dev_state(&st);
  if (rc) return rc;
  std::vector<BatchEntry> tab;
  std::vector<int64_t> big;
  tab.reserve((size_t)count);
  for (int64_t i = 0; i < count; ++i) {
    if (n[i] <= w) continue;  // already banded, no reflectors
    if (b <= batched_max_block() && n[i] - w <= batched_max_trailing() &&
        lda[i] * n[i] < ((int64_t)1 << 29))  // 32-bit element offsets in the kernel
      tab.push_back(BatchEntry{A[i], tau[i], lda[i], (int)n[i], 0});
    else
      big.push_back(i);
  }
  std::stable_sort(tab.begin(), tab.end(),
                   [](const BatchEntry &x, const BatchEntry &y) { return x.n > y.n; });
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  BR_HIP_CHECK(hipStreamIsCapturing(s, &cap));
  const bool capturing = cap != hipStreamCaptureStatusNone;
  if (!tab.empty()) {
    std::lock_guard<std::mutex> lk(g_mu);
    const int nwg = (int)std::min<int64_t>((int64_t)tab.size(), st->num_cu);
    const size_t tb = tab.size() * sizeof(BatchEntry);
    auto same_as = [&](const BatchTable &t) {
      return t.host.size() == tab.size() && memcmp(t.host.data(), tab.data(), tb) == 0;
    };
    BatchTable *table = nullptr;
    for (BatchTable &t : st->tables)
      if (same_as(t)) table = &t;
    if (capturing && (g_prof || !table || nwg > st->bt_wgs)) return BANDRED_ERR_UNSUPPORTED;
    if (!capturing) BR_HIP_CHECK(hipStreamWaitEvent(s, st->done, 0));
    if (nwg > st->bt_wgs) {
      BR_HIP_CHECK(hipEventSynchronize(st->done));
      if (st->bt_ws) {
        if (st->bt_ws_captured) st->retired.push_back(st->bt_ws);
        else BR_HIP_CHECK(hipFree(st->bt_ws));
      }
      st->bt_ws = nullptr;
      st->bt_wgs = 0;
      st->bt_ws_captured = false;
      if (hipMalloc((void **)&st->bt_ws, (size_t)nwg * batched_ws_doubles() * sizeof(double)) !=
          hipSuccess) {
        (void)hipGetLastError();
        st->bt_ws = nullptr;
        return BANDRED_ERR_ALLOC;
      }
      st->bt_wgs = nwg;
    }
    if (!table) {
      // reuse a table no captured graph refers to (the largest one that fits),
      // or add a new one; then upload through the pinned staging copy
      BR_HIP_CHECK(hipEventSynchronize(st->bt_ev));  // the staging copy is free again
      for (BatchTable &t : st->tables)
        if (!t.captured && t.cap >= tab.size() && (!table || t.cap > table->cap)) table = &t;
      if (table) {
        BR_HIP_CHECK(hipEventSynchronize(st->done));  // no kernel reads its old content
      } else {
        st->tables.emplace_back();
        table = &st->tables.back();
        table->cap = tab.size() + tab.size() / 4 + 64;
        if (hipMalloc((void **)&table->dev, table->cap * sizeof(BatchEntry)) != hipSuccess) {
          (void)hipGetLastError();
          st->tables.pop_back();
          return BANDRED_ERR_ALLOC;
        }
      }
      if (tab.size() > st->bt_stage_cap) {
        if (st->bt_stage) BR_HIP_CHECK(hipHostFree(st->bt_stage));
        st->bt_stage = nullptr;
        st->bt_stage_cap = 0;
        const size_t cap_e = tab.size() + tab.size() / 4 + 64;
        if (hipHostMalloc((void **)&st->bt_stage, cap_e * sizeof(BatchEntry),
                          hipHostMallocDefault) != hipSuccess) {
          (void)hipGetLastError();
          return BANDRED_ERR_ALLOC;
        }
        st->bt_stage_cap = cap_e;
      }
      table->host = tab;
      memcpy(st->bt_stage, tab.data(), tb);
      BR_HIP_CHECK(hipMemcpyAsync(table->dev, st->bt_stage, tb, hipMemcpyHostToDevice, s));
      BR_HIP_CHECK(hipEventRecord(st->bt_ev, s));
    }
    if (capturing) {
      table->captured = true;
      st->bt_ws_captured = true;
    }
    rc = launch_fill_u32(st->bt_queue, 1, 0u, s);
    if (rc) return rc;
    rc = launch_fill_u32((unsigned *)st->flags, 2, 0u, s);  // no bounded waits: stays 0
    if (rc) return rc;
    g_last_flags[current_dev_index()] = st->flags;
    double flops = 0.0;
    for (const BatchEntry &e : tab) flops += 4.0 / 3.0 * (double)e.n * e.n * e.n;
    {
      ProfScope ps(C_BATCHED, flops, s);
      rc = launch_batched(prec, table->dev, (int)tab.size(), w, b, st->bt_queue, st->bt_ws, nwg, s);
    }
    if (rc) return rc;
    if (!capturing) BR_HIP_CHECK(hipEventRecord(st->done, s));
  }
  if (!big.empty() && capturing) return BANDRED_ERR_UNSUPPORTED;
  for (int64_t i : big) {
    rc = sy2sb_impl(n[i], w, b, A[i], lda[i], tau[i], prec, nullptr, s);
    if (rc) return rc;
  }
  return 0;
}

// Device status word of the most recent call on the current device (0, or
// BANDRED_ERR_TIMEOUT), after the work on stream s has finished.
static int read_status(hipStream_t s) {
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  BR_HIP_CHECK(hipStreamSynchronize(s));
  if (!g_last_flags[dev]) return 0;  // no call on this device yet
  int flags[2] = {0, 0};
  BR_HIP_CHECK(hipMemcpy(flags, g_last_flags[dev], sizeof(flags), hipMemcpyDeviceToHost));
  return flags[0];
}

// ---------------------------------------------------------------------------
// No-allocation SY2SB.  The workspace is a fixed device array (one copy per
// device, alive until the process ends): the first 256 bytes hold the status
// words, the rest the arena that the library's own workspace would provide.
// Runs the serial order (no look-ahead stream, no events), so it can be
// called where allocation is impossible (under stream capture with no earlier
// eager call, or in loops that must not allocate).
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];

struct NoAllocDev {
  bool ready = false;
  DevState st;  // props, flags and arena inside the device copy of scratch
};
static NoAllocDev g_na[64];

// Device address of this device's copy of scratch (looked up once per device,
// with that device current), wrapped as a DevState without streams or events.
static int noalloc_state(DevState **out) {
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  NoAllocDev &na = g_na[dev];
  if (!na.ready) {
    rc = dev_props(na.st, dev);
    if (rc) return rc;
    void *p = nullptr;
    BR_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) return BANDRED_ERR_HIP;
    na.st.flags = reinterpret_cast<int *>(p);
    na.st.base = reinterpret_cast<char *>(p) + 256;
    na.st.bytes = kNoAllocBytes - 256;
    na.ready = true;
  }
  // the wait bound set by bandred_set_wait_limit_us applies here too
  if (g_dev[dev].props) na.st.timeout_ticks = g_dev[dev].timeout_ticks;
  *out = &na.st;
  return 0;
}

}  // namespace br

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace br;

static int check_sy2sb(int64_t n, int64_t w, int64_t b, const double *A, int64_t lda,
                       const double *tau) {
  if (n < 0) return -1;
  if (w < 1) return -2;
  if (b < 1 || b > w || b > kNbMax) return -3;
  if (n > 0 && A == nullptr) return -4;
  if (lda < (n > 1 ? n : 1)) return -5;
  if (n > w && tau == nullptr) return -6;
  return 0;
}

static int check_ge2gb(int64_t m, int64_t n, int64_t w, int64_t b, const double *A, int64_t lda,
                       const double *tauq, const double *taup) {
  if (m < 0) return -1;
  if (n < 0 || n > m) return (n < 0) ? -2 : -1;
  if (w < 1) return -3;
  if (b < 1 || b > w || b > kNbMax) return -4;
  if (n > 0 && A == nullptr) return -5;
  if (lda < (m > 1 ? m : 1)) return -6;
  if (n > 0 && tauq == nullptr) return -7;
  if (n > 0 && taup == nullptr) return -8;
  return 0;
}

static int check_prec(int prec) {
  return (prec == BANDRED_FP64 || prec == BANDRED_FP32_UPDATE || prec == BANDRED_SPLIT32_UPDATE ||
          prec == BANDRED_INT8_SPLIT_UPDATE)
             ? 0
             : 1;
}

static int check_opts(const bandred_opts_t *o) {
  if (!o) return 0;
  if (o->lookahead != 0 && o->lookahead != 1) return 1;
  if (o->panel_rows < 0) return 1;
  if (o->panel_method < 0 || o->panel_method > 2) return 1;
  if (o->update_chunks < 0 || o->update_chunks > 8) return 1;
  if (o->update_lds_cap < 0 || o->update_lds_cap > 2) return 1;
  for (int i = 0; i < 3; ++i)
    if (o->reserved[i] != 0) return 1;
  return 0;
}

// The options of a call that passed b = 0: the autotuner's knobs where the
// caller left them at 0.
static const bandred_opts_t *tuned_opts(const bandred_opts_t *opts, int chunks, int cap,
                                        bandred_opts_t *buf) {
  if (opts) *buf = *opts;
  else {
    *buf = bandred_opts_t{};
    buf->lookahead = 1;
  }
  if (buf->update_chunks == 0) buf->update_chunks = chunks;
  if (buf->update_lds_cap == 0) buf->update_lds_cap = cap;
  return buf;
}

extern "C" {

int bandred_sy2sb(int64_t n, int64_t w, int64_t b, double *A, int64_t lda, double *tau) {
  int rc = check_sy2sb(n, w, b, A, lda, tau);
  if (rc) return rc;
  rc = sy2sb_impl(n, w, b, A, lda, tau, BANDRED_FP64, nullptr, nullptr);
  if (rc) return rc;
  return read_status(nullptr);
}

int bandred_ge2gb(int64_t m, int64_t n, int64_t w, int64_t b, double *A, int64_t lda,
                  double *tauq, double *taup) {
  int rc = check_ge2gb(m, n, w, b, A, lda, tauq, taup);
  if (rc) return rc;
  rc = ge2gb_impl(m, n, w, b, A, lda, tauq, taup, BANDRED_FP64, nullptr, nullptr);
  if (rc) return rc;
  return read_status(nullptr);
}

int bandred_sy2sb_ex(int64_t n, int64_t w, int64_t b, double *A, int64_t lda, double *tau,
                     int prec, const bandred_opts_t *opts, void *stream) {
  int rc = check_sy2sb(n, w, b == 0 ? std::min<int64_t>(w, kNbMax) : b, A, lda, tau);
  if (rc) return rc;
  if (check_prec(prec)) return -7;
  if (check_opts(opts)) return -8;
  bandred_opts_t tuned;
  if (b == 0) {  // the autotuner's block size and update split
    int bt = 0;
    int ch = 0, cap = 0;
    rc = tune_pick(0, n, n, w, prec, (hipStream_t)stream, &bt, &ch, &cap);
    if (rc) return rc;
    b = bt;
    opts = tuned_opts(opts, ch, cap, &tuned);
  }
  return sy2sb_impl(n, w, b, A, lda, tau, prec, opts, (hipStream_t)stream);
}

int bandred_ge2gb_ex(int64_t m, int64_t n, int64_t w, int64_t b, double *A, int64_t lda,
                     double *tauq, double *taup, int prec, const bandred_opts_t *opts,
                     void *stream) {
  int rc = check_ge2gb(m, n, w, b == 0 ? std::min<int64_t>(w, kNbMax) : b, A, lda, tauq, taup);
  if (rc) return rc;
  if (check_prec(prec)) return -9;
  if (check_opts(opts)) return -10;
  bandred_opts_t tuned;
  if (b == 0) {
    int bt = 0;
    int ch = 0, cap = 0;
    rc = tune_pick(1, m, n, w, prec, (hipStream_t)stream, &bt, &ch, &cap);
    if (rc) return rc;
    b = bt;
    opts = tuned_opts(opts, ch, cap, &tuned);
  }
  return ge2gb_impl(m, n, w, b, A, lda, tauq, taup, prec, opts, (hipStream_t)stream);
}

int bandred_ge2gb_lu(int64_t m, int64_t n, int64_t w, int64_t b, double *A, int64_t lda,
                     double *tauq, double *taup, int prec, const bandred_opts_t *opts,
                     void *stream) {
  int rc = check_ge2gb(m, n, w, b == 0 ? std::min<int64_t>(w, kNbMax) : b, A, lda, tauq, taup);
  if (rc) return rc;
  if (check_prec(prec)) return -9;
  if (check_opts(opts)) return -10;
  bandred_opts_t tuned;
  if (b == 0) {
    int bt = 0;
    int ch = 0, cap = 0;
    rc = tune_pick(2, m, n, w, prec, (hipStream_t)stream, &bt, &ch, &cap);
    if (rc) return rc;
    b = bt;
    opts = tuned_opts(opts, ch, cap, &tuned);
  }
  return ge2gb_lu_impl(m, n, w, b, A, lda, tauq, taup, prec, opts, (hipStream_t)stream);
}

int bandred_sy2sb_apply_q(int trans, int64_t n, int64_t w, int64_t b, const double *A,
                          int64_t lda, const double *tau, int64_t k, double *C, int64_t ldc,
                          void *stream) {
  if (trans != 0 && trans != 1) return -1;
  if (n < 0) return -2;
  if (w < 1) return -3;
  if (b < 1 || b > kNbMax) return -4;
  const int64_t nrefl = n > w ? n - w : 0;
  if (nrefl > 0 && A == nullptr) return -5;
  if (lda < (n > 1 ? n : 1)) return -6;
  if (nrefl > 0 && tau == nullptr) return -7;
  if (k < 0) return -8;
  if (k > 0 && n > 0 && C == nullptr) return -9;
  if (ldc < (n > 1 ? n : 1)) return -10;
  return apply_impl(0, w, nrefl, n, A, lda, tau, trans, k, C, ldc, (int)b, (hipStream_t)stream);
}

int bandred_ge2gb_apply(int side, int form, int trans, int64_t m, int64_t n, int64_t w, int64_t b,
                        const double *A, int64_t lda, const double *tau, int64_t k, double *C,
                        int64_t ldc, void *stream) {
  if (side != 0 && side != 1) return -1;
  if (form != 0 && form != 1) return -2;
  if (trans != 0 && trans != 1) return -3;
  if (m < 0) return -4;
  if (n < 0 || n > m) return (n < 0) ? -5 : -4;
  if (w < 1) return -6;
  if (b < 1 || b > kNbMax) return -7;
  int64_t off, nrefl, len;
  if (side == 0) {  // U: column storage, m x k
    off = form ? w : 0;
    nrefl = form ? std::max<int64_t>(0, std::min<int64_t>(n, m - w)) : n;
    len = m;
  } else {          // V: row storage from column w on, n x k
    off = w;
    nrefl = std::max<int64_t>(0, n - w);
    len = n;
  }
  if (nrefl > 0 && A == nullptr) return -8;
  if (lda < (m > 1 ? m : 1)) return -9;
  if (nrefl > 0 && tau == nullptr) return -10;
  if (k < 0) return -11;
  if (k > 0 && len > 0 && C == nullptr) return -12;
  if (ldc < (len > 1 ? len : 1)) return -13;
  return apply_impl(side, off, nrefl, len, A, lda, tau, trans, k, C, ldc, (int)b,
                    (hipStream_t)stream);
}

int bandred_sb2st(int64_t n, int64_t w, const double *A, int64_t lda, double *d, double *e,
                  void *stream) {
  if (n < 0) return -1;
  if (w < 1) return -2;
  if (n > 0 && A == nullptr) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (n > 0 && d == nullptr) return -5;
  if (n > 1 && e == nullptr) return -6;
  return sb2st_impl(n, w, A, lda, d, e, (hipStream_t)stream);
}

int bandred_tridiag_eigvals(int64_t n, const double *d, const double *e, double *lam,
                            void *stream) {
  if (n < 0) return -1;
  if (n > 0 && d == nullptr) return -2;
  if (n > 1 && e == nullptr) return -3;
  if (n > 0 && lam == nullptr) return -4;
  return tridiag_eig_impl(n, d, e, lam, (hipStream_t)stream);
}

int bandred_sy2sb_noalloc(int64_t n, int64_t w, int64_t b, double *A, int64_t lda, double *tau,
                          int prec, void *stream) {
  int rc = check_sy2sb(n, w, b, A, lda, tau);
  if (rc) return rc;
  if (check_prec(prec)) return -7;
  DevState *na = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    rc = noalloc_state(&na);
  }
  if (rc) return rc;
  return sy2sb_impl(n, w, b, A, lda, tau, prec, nullptr, (hipStream_t)stream, na);
}

int bandred_sy2sb_batched(int64_t count, const int64_t *n, int64_t w, int64_t b, double *const *A,
                          const int64_t *lda, double *const *tau, int prec, void *stream) {
  if (count < 0) return -1;
  if (count > 0 && n == nullptr) return -2;
  if (w < 1) return -3;
  if (b < 1 || b > w || b > kNbMax) return -4;
  if (count > 0 && A == nullptr) return -5;
  if (count > 0 && lda == nullptr) return -6;
  if (count > 0 && tau == nullptr) return -7;
  if (prec != BANDRED_FP64 && prec != BANDRED_FP32_UPDATE) return -8;
  for (int64_t i = 0; i < count; ++i) {
    if (n[i] < 0) return -2;
    if (n[i] > 0 && A[i] == nullptr) return -5;
    if (lda[i] < (n[i] > 1 ? n[i] : 1)) return -6;
    if (n[i] > w && tau[i] == nullptr) return -7;
  }
  if (count == 0) return 0;
  if (w > ((int64_t)1 << 30)) return BANDRED_ERR_UNSUPPORTED;
  return batched_impl(count, n, (int)w, (int)b, A, lda, tau, prec, (hipStream_t)stream);
}

const char *bandred_status_string(int status) {
  switch (status) {
    case BANDRED_OK: return "success";
    case BANDRED_ERR_HIP: return "HIP runtime error";
    case BANDRED_ERR_ALLOC: return "device workspace allocation failed";
    case BANDRED_ERR_UNSUPPORTED: return "unsupported device or problem shape";
    case BANDRED_ERR_TIMEOUT: return "inter-workgroup wait timed out";
    default: break;
  }
  if (status < 0) return "invalid argument";
  return "unknown status";
}

int bandred_status(void *stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  return read_status((hipStream_t)stream);
}

int bandred_release(void) {
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState &st = g_dev[dev];
  if (!st.init) return 0;
  BR_HIP_CHECK(hipDeviceSynchronize());
  for (void *p : st.retired) BR_HIP_CHECK(hipFree(p));
  st.retired.clear();
  if (st.base) BR_HIP_CHECK(hipFree(st.base));
  st.base = nullptr;
  st.bytes = 0;
  st.base_captured = false;
  for (BatchTable &t : st.tables)
    if (t.dev) BR_HIP_CHECK(hipFree(t.dev));
  st.tables.clear();
  if (st.bt_stage) BR_HIP_CHECK(hipHostFree(st.bt_stage));
  st.bt_stage = nullptr;
  st.bt_stage_cap = 0;
  if (st.bt_ws) BR_HIP_CHECK(hipFree(st.bt_ws));
  st.bt_ws = nullptr;
  st.bt_wgs = 0;
  st.bt_ws_captured = false;
  return 0;
}

int bandred_set_wait_limit_us(double us) {
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState &st = g_dev[dev];
  rc = dev_props(st, dev);
  if (rc) return rc;
  // the wall clock runs at default_ticks / 10 s
  long long t = st.default_ticks;
  if (us > 0.0) {
    const double per_us = (double)st.default_ticks / 1e7;
    t = (long long)(us * per_us);
    if (t < 1) t = 1;
  }
  st.timeout_ticks = t;
  return 0;
}

int bandred_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof = on != 0;
  for (auto &r : g_prof_recs) {
    g_ev_pool.push_back(r.a);
    g_ev_pool.push_back(r.b);
  }
  g_prof_recs.clear();
  return 0;
}

int bandred_profile_read(double *out, int cap) {
  std::lock_guard<std::mutex> lk(g_mu);
  double acc[C_NCLS][3] = {};
  for (auto &r : g_prof_recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return -BANDRED_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return -BANDRED_ERR_HIP;
    acc[r.cls][0] += ms;
    acc[r.cls][1] += r.flops;
    acc[r.cls][2] += 1.0;
  }
  for (int c = 0; c < C_NCLS; ++c)
    for (int q = 0; q < 3; ++q)
      if (3 * c + q < cap) out[3 * c + q] = acc[c][q];
  for (auto &r : g_prof_recs) {
    g_ev_pool.push_back(r.a);
    g_ev_pool.push_back(r.b);
  }
  g_prof_recs.clear();
  return C_NCLS;
}

const char *bandred_profile_name(int cls) {
  if (cls < 0 || cls >= C_NCLS) return "";
  return kClsNames[cls];
}

}  // extern "C"
