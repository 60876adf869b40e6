// tune.hip -- autotuner of the reductions: block size and the split between
// the look-ahead panel and the update beside it.
//
// The paper tunes the algorithmic block size b per problem (n, w) in steps of
// 16 and shows that the best b depends on both (Sec. 4.2, the role of the
// block size; Table 1's b was picked that way).  The result of a reduction does
// not depend on b (up to rounding), only its speed does, so b can be chosen by
// timing: the tuner runs the reduction on a synthetic matrix of the same shape
// (values from a counter-based hash, so the timing sees no data-dependent
// fast path) for every candidate b in {16, 32, ..., min(w, 128)} (b = w when
// w < 16), and keeps the fastest.  At that b it then times the knobs that
// share the chip between the panel of the next step and the update beside it
// (the paper's split of the cores between panel and update, Sec. 2.2): the
// number of launches the update is issued as (1 .. 4) and whether they leave
// LDS room on each CU for the panel (on / off); these change no result bit,
// and a setting is kept when it beats the default rule by more than 1%.
// Results are cached per device and (kind, m, n, w, prec) in memory and, when
// the environment variable BANDRED_TUNE_CACHE names a file, in that file (one
// JSON object per line), which later processes read back.
//
// It is built only on the library's public entry points; it allocates the
// trial matrix and times with HIP events, so it must not run under stream
// capture.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace br {

// x -> a double in [-1, 1) from the 64-bit hash (splitmix64 finaliser) of
// the element's position and a seed
__device__ __forceinline__ double hash_unit(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// m x n column-major trial matrix; symmetric (element (i, j) hashed from
// (max, min)) when sym is set
__global__ void k_trial_fill(double *A, int64_t lda, int m, int n, int sym, uint64_t seed) {
  const int64_t total = (int64_t)m * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % m, j = idx / m;
    const int64_t a = sym ? std::max(i, j) : i, c = sym ? std::min(i, j) : j;
    A[i + j * lda] = hash_unit(seed ^ ((uint64_t)a * 0x100000001B3ull + (uint64_t)c));
  }
}

namespace {

struct TuneEntry {
  int dev, kind, prec;
  int64_t m, n, w;
  int b;
  int chunks, cap;  // bandred_opts_t.update_chunks / update_lds_cap (0: default rule)
};

std::mutex g_tmu;
std::vector<TuneEntry> g_cache;
bool g_file_read = false;

const char *kind_name(int kind) {
  return kind == 0 ? "sy2sb" : kind == 1 ? "ge2gb" : "ge2gb_lu";
}

// one line per entry: {"kind": "sy2sb", "m": M, "n": N, "w": W, "prec": P, "b": B, ...}
void read_file_locked() {
  if (g_file_read) return;
  g_file_read = true;
  const char *path = getenv("BANDRED_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  char line[1024], kname[32];
  while (fgets(line, sizeof line, f)) {
    long long m = 0, n = 0, w = 0;
    int prec = 0, b = 0;
    if (sscanf(line, " {\"kind\": \"%31[a-z0-9_]\", \"m\": %lld, \"n\": %lld, \"w\": %lld, "
                     "\"prec\": %d, \"b\": %d",
               kname, &m, &n, &w, &prec, &b) != 6)
      continue;
    int kind = -1;
    for (int k = 0; k < 3; ++k)
      if (strcmp(kname, kind_name(k)) == 0) kind = k;
    if (kind < 0 || b < 1 || b > kNbMax || b > w) continue;
    int chunks = 0, cap = 0;
    if (const char *q = strstr(line, "\"chunks\": ")) chunks = atoi(q + 10);
    if (const char *q = strstr(line, "\"cap\": ")) cap = atoi(q + 7);
    if (chunks < 0 || chunks > 8) chunks = 0;
    if (cap < 0 || cap > 2) cap = 0;
    g_cache.push_back(TuneEntry{-1, kind, prec, m, n, w, b, chunks, cap});  // any device
  }
  fclose(f);
}

void append_file(const TuneEntry &e, const std::vector<std::pair<int, float>> &times,
                 const std::vector<std::pair<int, float>> &split_times) {
  const char *path = getenv("BANDRED_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "{\"kind\": \"%s\", \"m\": %lld, \"n\": %lld, \"w\": %lld, \"prec\": %d, \"b\": %d, "
             "\"chunks\": %d, \"cap\": %d, \"ms\": {",
          kind_name(e.kind), (long long)e.m, (long long)e.n, (long long)e.w, e.prec, e.b, e.chunks,
          e.cap);
  for (size_t i = 0; i < times.size(); ++i)
    fprintf(f, "%s\"%d\": %.4f", i ? ", " : "", times[i].first, times[i].second);
  fprintf(f, "}, \"split_ms\": {");
  for (size_t i = 0; i < split_times.size(); ++i)  // key: 10 chunks + cap
    fprintf(f, "%s\"%d\": %.4f", i ? ", " : "", split_times[i].first, split_times[i].second);
  fprintf(f, "}}\n");
  fclose(f);
}

// the cached entry (nullptr when the problem has not been tuned)
const TuneEntry *lookup_locked(int dev, int kind, int64_t m, int64_t n, int64_t w, int prec) {
  read_file_locked();
  const TuneEntry *found = nullptr;
  for (const TuneEntry &e : g_cache)
    if ((e.dev == dev || e.dev < 0) && e.kind == kind && e.m == m && e.n == n && e.w == w &&
        e.prec == prec) {
      found = &e;
      if (e.dev == dev) return found;  // a measurement on this device wins
    }
  return found;
}

int run_once(int kind, int64_t m, int64_t n, int64_t w, int64_t b, double *A, int64_t lda,
             double *t1, double *t2, int prec, const bandred_opts_t *o, hipStream_t s) {
  if (kind == 0) return bandred_sy2sb_ex(n, w, b, A, lda, t1, prec, o, s);
  if (kind == 1) return bandred_ge2gb_ex(m, n, w, b, A, lda, t1, t2, prec, o, s);
  return bandred_ge2gb_lu(m, n, w, b, A, lda, t1, t2, prec, o, s);
}

}  // namespace

// Candidate block sizes for bandwidth w: multiples of 16 up to min(w, 128)
// (the paper's step), or w itself below 16.
static std::vector<int> candidates(int64_t w) {
  std::vector<int> c;
  const int top = (int)std::min<int64_t>(w, kNbMax);
  for (int b = 16; b <= top; b += 16) c.push_back(b);
  if (c.empty()) c.push_back(top);
  return c;
}

// Tuned b for the problem (kind 0: sy2sb n x n; 1: ge2gb m x n; 2: ge2gb_lu),
// measured now unless cached.  times (optional) receives the measured
// milliseconds per candidate.
int tune_block(int kind, int64_t m, int64_t n, int64_t w, int prec, int force, TuneEntry *out,
               std::vector<std::pair<int, float>> *times_out) {
  int dev = 0;
  BR_HIP_CHECK(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    const TuneEntry *e = force ? nullptr : lookup_locked(dev, kind, m, n, w, prec);
    if (e) {
      *out = *e;
      return 0;
    }
  }
  const std::vector<int> cand = candidates(w);
  if (kind == 0 ? n <= w + 1 : n == 0) {  // nothing to reduce: nothing to time
    *out = TuneEntry{dev, kind, prec, m, n, w, cand.back(), 0, 0};
    return 0;
  }
  const int64_t rows = (kind == 0) ? n : m;
  const int64_t lda = std::max<int64_t>(1, rows);
  const size_t elems = (size_t)lda * n;
  double *A0 = nullptr, *A = nullptr, *t1 = nullptr, *t2 = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t ea = nullptr, eb = nullptr;
  int rc = 0;
  std::vector<std::pair<int, float>> times;
  auto cleanup = [&]() {
    if (A0) (void)hipFree(A0);
    if (A) (void)hipFree(A);
    if (t1) (void)hipFree(t1);
    if (t2) (void)hipFree(t2);
    if (ea) (void)hipEventDestroy(ea);
    if (eb) (void)hipEventDestroy(eb);
    if (s) (void)hipStreamDestroy(s);
  };
  if (hipMalloc((void **)&A0, elems * 8) != hipSuccess || hipMalloc((void **)&A, elems * 8) != hipSuccess ||
      hipMalloc((void **)&t1, (size_t)std::max<int64_t>(n, 1) * 8) != hipSuccess ||
      hipMalloc((void **)&t2, (size_t)std::max<int64_t>(n, 1) * 8) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    return BANDRED_ERR_ALLOC;
  }
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess) {
    cleanup();
    return BANDRED_ERR_HIP;
  }
  hipLaunchKernelGGL(k_trial_fill, dim3(1024), dim3(256), 0, s, A0, lda, (int)rows, (int)n,
                     kind == 0 ? 1 : 0, (uint64_t)0x5EEDull);
  // best of two timed runs after a warm-up, each on a fresh copy of the matrix
  auto time_setting = [&](int b, const bandred_opts_t *o, float *ms_best) -> int {
    float tmin = 0.f;
    for (int rep = 0; rep < 3; ++rep) {
      if (hipMemcpyAsync(A, A0, elems * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return BANDRED_ERR_HIP;
      (void)hipEventRecord(ea, s);
      const int r = run_once(kind, m, n, w, b, A, lda, t1, t2, prec, o, s);
      (void)hipEventRecord(eb, s);
      if (r) return r;
      if (hipEventSynchronize(eb) != hipSuccess) return BANDRED_ERR_HIP;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ea, eb);
      if (rep > 0 && (tmin == 0.f || ms < tmin)) tmin = ms;
    }
    *ms_best = tmin;
    return 0;
  };
  // (1) the block size, with the default split
  float best = 0.f;
  int bbest = cand.back();
  for (int b : cand) {
    if (cand.size() == 1) break;
    float t = 0.f;
    rc = time_setting(b, nullptr, &t);
    if (rc) break;
    times.emplace_back(b, t);
    if (best == 0.f || t < best) {
      best = t;
      bbest = b;
    }
  }
  // (2) at that b, the update's launches and LDS cap beside the panel
  int cbest = 0, lbest = 0;
  std::vector<std::pair<int, float>> split_times;
  if (rc == 0 && best == 0.f) rc = time_setting(bbest, nullptr, &best);
  float sbest = best;
  for (int ch = 1; ch <= 4 && rc == 0; ++ch)
    for (int cap = 1; cap <= 2 && rc == 0; ++cap) {
      bandred_opts_t o{};
      o.lookahead = 1;
      o.update_chunks = ch;
      o.update_lds_cap = cap;
      float t = 0.f;
      rc = time_setting(bbest, &o, &t);
      if (rc) break;
      split_times.emplace_back(10 * ch + cap, t);
      if (t < sbest) {
        sbest = t;
        cbest = ch;
        lbest = cap;
      }
    }
  if (sbest > 0.99f * best) cbest = lbest = 0;  // within 1% of the default: keep it
  if (rc == 0 && hipStreamSynchronize(s) != hipSuccess) rc = BANDRED_ERR_HIP;
  if (rc == 0) rc = bandred_status(s);
  cleanup();
  if (rc) return rc;
  TuneEntry e{dev, kind, prec, m, n, w, bbest, cbest, lbest};
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_cache.push_back(e);
    append_file(e, times, split_times);
  }
  *out = e;
  if (times_out) *times_out = times;
  return 0;
}

// Cached b only (0 when the problem has not been tuned).
int tune_lookup(int kind, int64_t m, int64_t n, int64_t w, int prec) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(g_tmu);
  const TuneEntry *e = lookup_locked(dev, kind, m, n, w, prec);
  return e ? e->b : 0;
}

}  // namespace br

using namespace br;

extern "C" int bandred_tune(int kind, int64_t m, int64_t n, int64_t w, int prec, int force,
                            int64_t *b_out, double *ms_out, int cap) {
  if (kind < 0 || kind > 2) return -1;
  if (m < 0) return -2;
  if (n < 0 || (kind != 0 && n > m)) return -3;
  if (w < 1) return -4;
  if (prec < 0 || prec > 3) return -5;
  if (b_out == nullptr) return -7;
  if (kind == 0) m = n;
  TuneEntry e{};
  std::vector<std::pair<int, float>> times;
  const int rc = tune_block(kind, m, n, w, prec, force, &e, &times);
  if (rc) return rc;
  *b_out = e.b;
  if (ms_out)
    for (int i = 0; i < cap; ++i) {
      ms_out[2 * i] = 0.0;
      ms_out[2 * i + 1] = 0.0;
      if (i < (int)times.size()) {
        ms_out[2 * i] = times[i].first;
        ms_out[2 * i + 1] = times[i].second;
      }
    }
  return 0;
}

extern "C" int bandred_tune_result(int kind, int64_t m, int64_t n, int64_t w, int prec,
                                   int64_t *b, int *update_chunks, int *update_lds_cap) {
  if (kind < 0 || kind > 2) return -1;
  if (kind == 0) m = n;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BANDRED_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_tmu);
  const TuneEntry *e = lookup_locked(dev, kind, m, n, w, prec);
  if (!e) return BANDRED_ERR_UNSUPPORTED;
  if (b) *b = e->b;
  if (update_chunks) *update_chunks = e->chunks;
  if (update_lds_cap) *update_lds_cap = e->cap;
  return 0;
}

namespace br {
// b and the update split for a call that passed b = 0: the cached choice,
// else (outside stream capture) a fresh measurement.
int tune_pick(int kind, int64_t m, int64_t n, int64_t w, int prec, hipStream_t s, int *b_out,
              int *chunks, int *cap) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  BR_HIP_CHECK(hipStreamIsCapturing(s, &cs));
  TuneEntry e{};
  if (cs != hipStreamCaptureStatusNone) {
    int dev = 0;
    BR_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tmu);
    const TuneEntry *c = lookup_locked(dev, kind, m, n, w, prec);
    if (!c) return BANDRED_ERR_UNSUPPORTED;  // cannot measure under capture
    e = *c;
  } else {
    const int rc = tune_block(kind, m, n, w, prec, 0, &e, nullptr);
    if (rc) return rc;
  }
  *b_out = e.b;
  *chunks = e.chunks;
  *cap = e.cap;
  return 0;
}
}  // namespace br
