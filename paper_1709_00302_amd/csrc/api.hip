// api.hip -- C ABI, workspace and the blocked drivers of the band reductions.
//
// SY2SB driver (Sec. 2.1; look-ahead Variant V2 of Sec. 2.2 when 2b > w and
// the V1 partition when 2b <= w).  Per panel c (width pb, r = c + w,
// j = n - r):
//   1. panel QR of A0 = A[r:n, c:c+pb]  -> V (explicit), tau, in-place R/v
//      (eq. updateA0)
//   2. S = V^T V, T = larft(S, tau)      (compact WY, Q = I - V T V^T)
//   3. A1 -= V T^T (V^T A1) on the w-pb in-band columns right of the panel
//      (eq. updateA1; empty when b = w)
//   4. P = A2 V (SYMM), X = P T          (eq. updateA2symm with W_paper = -V T)
//   5. M = T^T (V^T X), W = X - 1/2 V M  (eqs. updateA2gemm1/gemm2, X3 = -W)
//   6. A2 -= W V^T + V W^T (SYR2K, lower triangle; eq. updateA2syr2k)
// With look-ahead, step 6 is split: first the columns of A2 that belong to the
// next panel (A2^L), then -- while the next panel is factored on a second
// stream -- the rest (A2^R).
//
// GE2GB driver (Sec. 3.1, triangular-band form, b <= w).  Per block c:
//   1. left QR of A[c:m, c:c+pb]                (eq. updateB)
//   2. E = A[c:m, c+pb:n]: E -= V T^T (V^T E)    (eq. updateCD)
//   3. right LQ of A[c:c+pr, c+w:n]             (eq. updateC)
//   4. D = A[c+pr:m, c+w:n]: D -= (D U) T U^T    (eq. updateD)
#include <mutex>
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
enum Cls { C_PANEL = 0, C_LARFT, C_SYMM, C_SYR2K, C_GEMM_SMALL, C_REDUCE, C_GEMM_UPD, C_OTHER, C_NCLS };
static const char *kClsNames[C_NCLS] = {"panel_qr", "larft", "symm", "syr2k",
                                        "gemm_small", "reduce", "gemm_update", "other"};
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
struct DevState {
  bool init = false;
  char *base = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;  // completion of the previous call's work
  hipStream_t aux = nullptr;  // look-ahead (panel) stream
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  int *flags = nullptr;       // [0] status, [1] abort   (device)
  long long timeout_ticks = 0;
  int num_cu = 0;
};
static std::mutex g_mu;
static DevState g_dev[64];

static int dev_state(DevState **out) {
  int dev = 0;
  BR_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return BANDRED_ERR_UNSUPPORTED;
  DevState &st = g_dev[dev];
  if (!st.init) {
    hipDeviceProp_t prop;
    BR_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return BANDRED_ERR_UNSUPPORTED;
    st.num_cu = prop.multiProcessorCount;
    int rate_khz = 0;
    BR_HIP_CHECK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
    if (rate_khz <= 0) rate_khz = 100000;
    st.timeout_ticks = (long long)rate_khz * 1000LL * 10LL;  // 10 s per wait
    BR_HIP_CHECK(hipEventCreateWithFlags(&st.done, hipEventDisableTiming));
    BR_HIP_CHECK(hipEventCreateWithFlags(&st.ev_a, hipEventDisableTiming));
    BR_HIP_CHECK(hipEventCreateWithFlags(&st.ev_b, hipEventDisableTiming));
    BR_HIP_CHECK(hipStreamCreateWithFlags(&st.aux, hipStreamNonBlocking));
    BR_HIP_CHECK(hipMalloc((void **)&st.flags, 64));
    BR_HIP_CHECK(hipMemset(st.flags, 0, 64));
    BR_HIP_CHECK(hipEventRecord(st.done, st.aux));
    st.init = true;
  }
  *out = &st;
  return 0;
}

// Grow the workspace to at least `bytes`; waits for the previous call first.
static int ws_reserve(DevState &st, size_t bytes) {
  if (bytes <= st.bytes) return 0;
  BR_HIP_CHECK(hipEventSynchronize(st.done));
  if (st.base) BR_HIP_CHECK(hipFree(st.base));
  st.base = nullptr;
  st.bytes = 0;
  const size_t want = bytes + (bytes >> 3);
  if (hipMalloc((void **)&st.base, want) != hipSuccess) {
    (void)hipGetLastError();
    st.base = nullptr;
    return BANDRED_ERR_ALLOC;
  }
  st.bytes = want;
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
};

// C(M x N) = alpha op(A) op(B) + beta C, split over k when that fills the chip.
static int gemm(Ctx &cx, int cls, int opa, int opb, int prec, int M, int N, int K,
                const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                int64_t ldc, double alpha, double beta, hipStream_t s) {
  if (M <= 0 || N <= 0) return 0;
  if (K <= 0) {
    if (beta == 1.0) return 0;
    return BANDRED_ERR_UNSUPPORTED;  // never needed by the drivers
  }
  GemmDesc d{};
  d.M = M; d.N = N; d.K = K;
  d.A = A; d.lda = lda; d.B = B; d.ldb = ldb; d.C = C; d.ldc = ldc;
  d.alpha = alpha; d.beta = beta;
  const int bm = (M <= 64 && N <= 64) ? 64 : 128;
  const int tiles = ((M + bm - 1) / bm) * ((N + bm - 1) / bm);
  const int target = 2 * cx.st->num_cu;
  int ks = 1;
  if (tiles < target && K > 512) {
    ks = (target + tiles - 1) / tiles;
    const int maxks = K / 256;
    if (ks > maxks) ks = maxks;
    if (ks < 1) ks = 1;
    while (ks > 1 && (size_t)ks * M * N > cx.part_cap) --ks;
  }
  const double flops = 2.0 * M * N * (double)K;
  if (ks == 1) {
    d.kchunk = (int)round_up(K, kBK);
    ProfScope ps(cls, flops, s);
    return launch_gemm(opa, opb, E_AXPBY, prec, d, 1, s);
  }
  d.kchunk = (int)round_up((K + ks - 1) / ks, 128);
  ks = (K + d.kchunk - 1) / d.kchunk;
  d.part = cx.part;
  {
    ProfScope ps(cls, flops, s);
    int rc = launch_gemm(opa, opb, E_PART, prec, d, ks, s);
    if (rc) return rc;
  }
  ProfScope ps(C_REDUCE, 0.0, s);
  return launch_reduce_partials(cx.part, ks, M, N, alpha, C, ldc, beta, s);
}

// A2(lower, columns [c0, c1)) -= W V^T + V W^T with WV = [W | V] (j x 2pb).
static int syr2k(Ctx &cx, int prec, int j, int pb, const double *WV, int64_t ldwv, double *A2,
                 int64_t lda, int c0, int c1, hipStream_t s) {
  if (c1 <= c0) return 0;
  GemmDesc d{};
  d.M = j; d.N = j; d.K = 2 * pb;
  d.A = WV; d.lda = ldwv; d.B = WV; d.ldb = ldwv;
  d.C = A2; d.ldc = lda;
  d.rot = pb; d.c0 = c0; d.c1 = c1;
  d.kchunk = 2 * pb;
  // lower-trapezoid flops of the column range
  const double rows0 = (double)(j - c0), rows1 = (double)(j - c1);
  const double elems = 0.5 * (rows0 * (rows0 + 1) - rows1 * (rows1 + 1));
  ProfScope ps(C_SYR2K, 2.0 * 2.0 * pb * elems, s);
  return launch_gemm(A_N, B_TROT, E_SYR2K, prec, d, 1, s);
}

static int panel(Ctx &cx, bool rowmajor, double *P, int64_t ldp, int m, int nb, double *V,
                 int64_t ldv, double *tau, double *part2, double *piv, unsigned *counter,
                 int panel_rows, hipStream_t s) {
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
  d.part = part2; d.piv = piv; d.counter = counter;
  d.status = st.flags; d.abort_flag = st.flags + 1;
  d.timeout_ticks = st.timeout_ticks;
  ProfScope ps(C_PANEL, 2.0 * (double)m * nb * nb, s);
  return launch_panel(rowmajor, d, nwg, s);
}

// ---------------------------------------------------------------------------
// SY2SB
// ---------------------------------------------------------------------------
static int sy2sb_impl(int64_t n64, int64_t w64, int64_t b64, double *A, int64_t lda, double *tau,
                      int prec, const bandred_opts_t *opts, hipStream_t s) {
  if (n64 <= w64 + 1) {
    if (n64 > w64) {
      // one trivial reflector of length 1
      return launch_fill(tau, n64 - w64, 0.0, s);
    }
    return 0;
  }
  if (n64 > (int64_t)1 << 30) return BANDRED_ERR_UNSUPPORTED;
  const int n = (int)n64, w = (int)w64, b = (int)b64;
  const int lookahead = opts ? opts->lookahead : 1;
  const int panel_rows = opts ? opts->panel_rows : 0;
  DevState *st = nullptr;
  int rc = dev_state(&st);
  if (rc) return rc;

  const int nref = n - w - 1;               // reflector columns 0 .. n-w-2
  const int npan = (nref + b - 1) / b;
  const int jmax = n - w;                    // rows of the first panel
  const size_t part_cap = std::max<size_t>((size_t)8 * jmax * b, (size_t)256 * b * b);
  size_t need = 0;
  need += 2 * round_up((size_t)jmax * 2 * b * 8, 256);        // WV[2]
  need += round_up((size_t)jmax * b * 8, 256);                // P
  need += round_up(part_cap * 8, 256);                        // split-k partials
  need += 6 * round_up((size_t)b * std::max(b, w) * 8, 256);  // S T Y M Z Z2
  need += round_up((size_t)2 * 256 * kNbMax * 8, 256);        // panel partials
  need += round_up((size_t)kNbMax * kNbMax * 8, 256);         // pivot rows
  need += round_up((size_t)(npan + 1) * 4, 256);              // counters
  need += 4096;
  std::lock_guard<std::mutex> lk(g_mu);
  rc = ws_reserve(*st, need);
  if (rc) return rc;
  Arena ar(st->base);
  double *WVbuf[2] = {ar.take<double>((size_t)jmax * 2 * b), ar.take<double>((size_t)jmax * 2 * b)};
  double *Pb = ar.take<double>((size_t)jmax * b);
  double *part = ar.take<double>(part_cap);
  const size_t sq = (size_t)b * std::max(b, w);
  double *Sb = ar.take<double>(sq), *Tb[2] = {ar.take<double>(sq), ar.take<double>(sq)};
  double *Yb = ar.take<double>(sq), *Mb = ar.take<double>(sq), *Zb = ar.take<double>(sq);
  double *Z2b = ar.take<double>(sq);
  double *part2 = ar.take<double>((size_t)2 * 256 * kNbMax);
  double *piv = ar.take<double>((size_t)kNbMax * kNbMax);
  unsigned *counters = ar.take<unsigned>(npan + 1);

  Ctx cx{st, s, part, part_cap};
  hipStream_t ps = lookahead ? st->aux : s;  // panel stream

  // order after the previous call, reset flags and counters
  BR_HIP_CHECK(hipStreamWaitEvent(s, st->done, 0));
  rc = launch_fill_u32(counters, npan + 1, 0u, s); if (rc) return rc;
  rc = launch_fill_u32((unsigned *)st->flags, 2, 0u, s); if (rc) return rc;
  rc = launch_fill(tau, n - w, 0.0, s); if (rc) return rc;

  // prologue: panel 0 on the main stream
  {
    const int pb = std::min(b, nref);
    const int r = w, j = n - r;
    double *V = WVbuf[0] + (int64_t)pb * j;
    rc = panel(cx, false, A + r, lda, j, pb, V, j, tau, part2, piv, counters, panel_rows, s);
    if (rc) return rc;
    rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, P_F64, pb, pb, j, V, j, V, j, Sb, pb, 1.0, 0.0, s);
    if (rc) return rc;
    { ProfScope p2(C_LARFT, 0.0, s); rc = launch_larft(Sb, pb, tau, pb, Tb[0], pb, s); }
    if (rc) return rc;
  }

  for (int it = 0, c = 0; c < nref; ++it, c += b) {
    const int pb = std::min(b, nref - c);
    const int r = c + w, j = n - r;
    double *WV = WVbuf[it & 1];
    double *W = WV, *V = WV + (int64_t)pb * j;
    double *T = Tb[it & 1];
    double *A2 = A + r + (int64_t)r * lda;

    // next panel geometry
    const int cn = c + b;
    const bool has_next = cn < nref;
    const int pbn = has_next ? std::min(b, nref - cn) : 0;
    const int rn = cn + w, jn = n - rn;
    // columns of the next panel inside A1 ([cn, r)) and inside A2 ([r, cn+pbn))
    const int nxt_a1_lo = cn, nxt_a1_hi = std::min(cn + pbn, r);
    const int a2L = has_next ? std::max(0, cn + pbn - r) : 0;  // A2 columns the next panel needs

    // (3) left update of A1 = A[r:n, c+pb : r]
    const int a1w = w - pb;
    if (a1w > 0) {
      double *A1 = A + r + (int64_t)(c + pb) * lda;
      rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, P_F64, pb, a1w, j, V, j, A1, lda, Zb, pb, 1.0, 0.0, s);
      if (rc) return rc;
      rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, P_F64, pb, a1w, pb, T, pb, Zb, pb, Z2b, pb, 1.0, 0.0, s);
      if (rc) return rc;
      rc = gemm(cx, C_GEMM_UPD, A_N, B_N, prec, j, a1w, pb, V, j, Z2b, pb, A1, lda, -1.0, 1.0, s);
      if (rc) return rc;
    }
    (void)nxt_a1_lo; (void)nxt_a1_hi;
    // (4) P = A2 V ; X = P T  (X stored in W's slot)
    rc = gemm(cx, C_SYMM, A_SYM, B_N, prec, j, pb, j, A2, lda, V, j, Pb, j, 1.0, 0.0, s);
    if (rc) return rc;
    rc = gemm(cx, C_GEMM_SMALL, A_N, B_N, P_F64, j, pb, pb, Pb, j, T, pb, W, j, 1.0, 0.0, s);
    if (rc) return rc;
    // (5) Y = V^T X ; M = T^T Y ; W = X - 1/2 V M
    rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, P_F64, pb, pb, j, V, j, W, j, Yb, pb, 1.0, 0.0, s);
    if (rc) return rc;
    rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, P_F64, pb, pb, pb, T, pb, Yb, pb, Mb, pb, 1.0, 0.0, s);
    if (rc) return rc;
    rc = gemm(cx, C_GEMM_SMALL, A_N, B_N, P_F64, j, pb, pb, V, j, Mb, pb, W, j, -0.5, 1.0, s);
    if (rc) return rc;
    // (6) SYR2K: A2^L first, then the next panel (look-ahead) overlapped with A2^R
    rc = syr2k(cx, prec, j, pb, WV, j, A2, lda, 0, a2L, s);
    if (rc) return rc;
    if (has_next) {
      if (ps != s) {
        BR_HIP_CHECK(hipEventRecord(st->ev_a, s));
        BR_HIP_CHECK(hipStreamWaitEvent(ps, st->ev_a, 0));
      }
      double *WVn = WVbuf[(it + 1) & 1];
      double *Vn = WVn + (int64_t)pbn * jn;
      double *Tn = Tb[(it + 1) & 1];
      rc = panel(cx, false, A + rn + (int64_t)cn * lda, lda, jn, pbn, Vn, jn, tau + cn, part2, piv,
                 counters + it + 1, panel_rows, ps);
      if (rc) return rc;
      rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, P_F64, pbn, pbn, jn, Vn, jn, Vn, jn, Sb, pbn, 1.0, 0.0,
                ps);
      if (rc) return rc;
      { ProfScope p2(C_LARFT, 0.0, ps); rc = launch_larft(Sb, pbn, tau + cn, pbn, Tn, pbn, ps); }
      if (rc) return rc;
    }
    rc = syr2k(cx, prec, j, pb, WV, j, A2, lda, a2L, j, s);
    if (rc) return rc;
    if (has_next && ps != s) {
      BR_HIP_CHECK(hipEventRecord(st->ev_b, ps));
      BR_HIP_CHECK(hipStreamWaitEvent(s, st->ev_b, 0));
    }
  }
  BR_HIP_CHECK(hipEventRecord(st->done, s));
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
  DevState *st = nullptr;
  int rc = dev_state(&st);
  if (rc) return rc;
  const int npan = (n + b - 1) / b;
  const size_t part_cap = std::max<size_t>((size_t)8 * m * b, (size_t)256 * b * b);
  size_t need = 0;
  need += round_up((size_t)m * b * 8, 256);           // V (left)
  need += round_up((size_t)n * b * 8, 256);           // U (right)
  need += round_up((size_t)b * n * 8, 256) * 2;       // Z, Z2 (b x n)
  need += round_up((size_t)m * b * 8, 256) * 2;       // X, X2 (m x b)
  need += round_up(part_cap * 8, 256);
  need += 3 * round_up((size_t)b * b * 8, 256);       // S, Tq, Tp
  need += round_up((size_t)2 * 256 * kNbMax * 8, 256);
  need += round_up((size_t)kNbMax * kNbMax * 8, 256);
  need += round_up((size_t)(2 * npan + 2) * 4, 256);
  need += 4096;
  std::lock_guard<std::mutex> lk(g_mu);
  rc = ws_reserve(*st, need);
  if (rc) return rc;
  Arena ar(st->base);
  double *Vq = ar.take<double>((size_t)m * b);
  double *Up = ar.take<double>((size_t)n * b);
  double *Zb = ar.take<double>((size_t)b * n), *Z2b = ar.take<double>((size_t)b * n);
  double *Xb = ar.take<double>((size_t)m * b), *X2b = ar.take<double>((size_t)m * b);
  double *part = ar.take<double>(part_cap);
  double *Sb = ar.take<double>((size_t)b * b), *Tq = ar.take<double>((size_t)b * b);
  double *Tp = ar.take<double>((size_t)b * b);
  double *part2 = ar.take<double>((size_t)2 * 256 * kNbMax);
  double *piv = ar.take<double>((size_t)kNbMax * kNbMax);
  unsigned *counters = ar.take<unsigned>(2 * npan + 2);
  Ctx cx{st, s, part, part_cap};

  BR_HIP_CHECK(hipStreamWaitEvent(s, st->done, 0));
  rc = launch_fill_u32(counters, 2 * npan + 2, 0u, s); if (rc) return rc;
  rc = launch_fill_u32((unsigned *)st->flags, 2, 0u, s); if (rc) return rc;
  rc = launch_fill(tauq, n, 0.0, s); if (rc) return rc;
  rc = launch_fill(taup, n, 0.0, s); if (rc) return rc;

  for (int it = 0, c = 0; c < n; ++it, c += b) {
    const int pb = std::min(b, n - c);
    const int i = m - c;
    // (1) left panel QR of A[c:m, c:c+pb]
    rc = panel(cx, false, A + c + (int64_t)c * lda, lda, i, pb, Vq, i, tauq + c, part2, piv,
               counters + 2 * it, panel_rows, s);
    if (rc) return rc;
    rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, P_F64, pb, pb, i, Vq, i, Vq, i, Sb, pb, 1.0, 0.0, s);
    if (rc) return rc;
    { ProfScope p2(C_LARFT, 0.0, s); rc = launch_larft(Sb, pb, tauq + c, pb, Tq, pb, s); }
    if (rc) return rc;
    // (2) E = A[c:m, c+pb:n] -= V T^T (V^T E)
    const int ne = n - c - pb;
    if (ne > 0) {
      double *E = A + c + (int64_t)(c + pb) * lda;
      rc = gemm(cx, C_GEMM_UPD, A_T, B_N, prec, pb, ne, i, Vq, i, E, lda, Zb, pb, 1.0, 0.0, s);
      if (rc) return rc;
      rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, P_F64, pb, ne, pb, Tq, pb, Zb, pb, Z2b, pb, 1.0, 0.0, s);
      if (rc) return rc;
      rc = gemm(cx, C_GEMM_UPD, A_N, B_N, prec, i, ne, pb, Vq, i, Z2b, pb, E, lda, -1.0, 1.0, s);
      if (rc) return rc;
    }
    // (3) right LQ of the rows c .. c+pr-1 that own a right reflector
    const int pr = std::max(0, std::min(pb, n - w - 1 - c));
    if (pr > 0) {
      const int c0 = c + w, jr = n - c0;
      rc = panel(cx, true, A + c + (int64_t)c0 * lda, lda, jr, pr, Up, jr, taup + c, part2, piv,
                 counters + 2 * it + 1, panel_rows, s);
      if (rc) return rc;
      rc = gemm(cx, C_GEMM_SMALL, A_T, B_N, P_F64, pr, pr, jr, Up, jr, Up, jr, Sb, pr, 1.0, 0.0, s);
      if (rc) return rc;
      { ProfScope p2(C_LARFT, 0.0, s); rc = launch_larft(Sb, pr, taup + c, pr, Tp, pr, s); }
      if (rc) return rc;
      // (4) D = A[c+pr:m, c0:n]: X = D U ; X2 = X T ; D -= X2 U^T
      const int md = m - c - pr;
      if (md > 0) {
        double *D = A + (c + pr) + (int64_t)c0 * lda;
        rc = gemm(cx, C_GEMM_UPD, A_N, B_N, prec, md, pr, jr, D, lda, Up, jr, Xb, md, 1.0, 0.0, s);
        if (rc) return rc;
        rc = gemm(cx, C_GEMM_SMALL, A_N, B_N, P_F64, md, pr, pr, Xb, md, Tp, pr, X2b, md, 1.0, 0.0, s);
        if (rc) return rc;
        rc = gemm(cx, C_GEMM_UPD, A_N, B_T, prec, md, jr, pr, X2b, md, Up, jr, D, lda, -1.0, 1.0, s);
        if (rc) return rc;
      }
    }
  }
  BR_HIP_CHECK(hipEventRecord(st->done, s));
  return 0;
}

static int read_status(hipStream_t s) {
  DevState *st = nullptr;
  int rc = dev_state(&st);
  if (rc) return rc;
  int flags[2] = {0, 0};
  BR_HIP_CHECK(hipMemcpyAsync(flags, st->flags, sizeof(flags), hipMemcpyDeviceToHost, s));
  BR_HIP_CHECK(hipStreamSynchronize(s));
  return flags[0];
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
  return (prec == BANDRED_FP64 || prec == BANDRED_FP32_UPDATE || prec == BANDRED_SPLIT32_UPDATE)
             ? 0
             : 1;
}

static int check_opts(const bandred_opts_t *o) {
  if (!o) return 0;
  if (o->lookahead != 0 && o->lookahead != 1) return 1;
  if (o->panel_rows < 0) return 1;
  for (int i = 0; i < 6; ++i)
    if (o->reserved[i] != 0) return 1;
  return 0;
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
  int rc = check_sy2sb(n, w, b, A, lda, tau);
  if (rc) return rc;
  if (check_prec(prec)) return -7;
  if (check_opts(opts)) return -8;
  return sy2sb_impl(n, w, b, A, lda, tau, prec, opts, (hipStream_t)stream);
}

int bandred_ge2gb_ex(int64_t m, int64_t n, int64_t w, int64_t b, double *A, int64_t lda,
                     double *tauq, double *taup, int prec, const bandred_opts_t *opts,
                     void *stream) {
  int rc = check_ge2gb(m, n, w, b, A, lda, tauq, taup);
  if (rc) return rc;
  if (check_prec(prec)) return -9;
  if (check_opts(opts)) return -10;
  return ge2gb_impl(m, n, w, b, A, lda, tauq, taup, prec, opts, (hipStream_t)stream);
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
  (void)stream;
  return BANDRED_ERR_UNSUPPORTED;
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
