// tune.hip -- the autotuner: measures the schedule and tile choices that do
// not change any result and records the fastest for this process.
//
// * Search choice (lbdd_tune_search).  A refinement search that may run in
//   Dijkstra order runs so when the Bellman-Ford rounds it would need (a
//   running mean) cost more than the Dijkstra steps it would need (another
//   running mean), a round costing `ratio` steps.  By default the solve
//   measures the ratio itself from the device times of both kinds; the
//   candidates are that automatic ratio, always Bellman-Ford (0), a fixed
//   ratio (4 steps) and Dijkstra whenever the potentials allow it (2^20).
//   The tuner solves (a prefix of) the caller's instance once per candidate
//   and keeps the fastest, if it beats the default by more than 2 %;
//   instances created afterwards with the same k start with it
//   (lbdd_set_option overrides it per instance), and so do the instances of
//   a batched launch, which read it from their own state.
// * Scan tiles (lbdd_tune_best_transfers).  The whole-matrix scan can give a
//   row 1 to 64 lanes, each lane 1 to 32 column groups, and run one or two
//   resident waves of workgroups.  The tuner times every shape that fits k on
//   the caller's inputs; later scans with the same k and load width use the
//   fastest, if it beats the default by more than 2 %.
// Every candidate computes the same bits (searches: the same labels,
// predecessors and hops; the scan: keys reduced by an exact minimum), so the
// tuned choice is a matter of time only.
#include <hip/hip_runtime.h>

#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/lbdd.h"
#include "instance.hpp"
#include "lbdd_dev.hpp"
#include "tune_cache.hpp"

namespace lbdd {
namespace {
std::mutex g_mu;
std::map<std::pair<int, int>, int64_t> g_ratio;   // (k bucket, n bucket) -> search ratio (x16)
std::once_flag g_autoload;
}  // namespace

int tune_bucket_k(int32_t k) {
  int b = 0;
  while (k > 0) { ++b; k >>= 1; }
  return b;                                       // k in [2^(b-1), 2^b)
}

int tune_bucket_n(int64_t n) {
  int b = 0;
  while (n >= 10) { ++b; n /= 10; }
  return b;                                       // n in [10^b, 10^(b+1))
}

int64_t tuned_search_ratio(int32_t k, int64_t n) {
  tune_cache_autoload();
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_ratio.find({tune_bucket_k(k), tune_bucket_n(n)});
  return it == g_ratio.end() ? DEFAULT_SEARCH_RATIO : it->second;
}

// The tuning cache named by LBDD_TUNE_CACHE, read once per process on the
// first lookup (for this device's architecture); a missing or unreadable
// file leaves the defaults, and the caller's last error is kept.
void tune_cache_autoload() {
  std::call_once(g_autoload, [] {
    const char *path = std::getenv("LBDD_TUNE_CACHE");
    if (!path || !*path) return;
    const std::string saved = g_err;
    (void)lbdd_tune_load(path, nullptr);
    g_err = saved;
  });
}
}  // namespace lbdd

namespace {
using lbdd::fail;

// a candidate replaces the default only if it is faster by more than 2 %
constexpr float NOISE = 0.98f;

int hip_err(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? LBDD_E_NOMEM : LBDD_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// elapsed milliseconds of the work between two events on one stream
struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t init() {
    hipError_t e = hipEventCreate(&a);
    return e == hipSuccess ? hipEventCreate(&b) : e;
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};
}  // namespace

extern "C" {

int lbdd_tune_search(int32_t k, int64_t n, const int32_t *cm, const int32_t *capacity,
                     const int32_t *penalty, uint32_t flags, int64_t iters, void *hip_stream,
                     int64_t *ratio_out, float *ms_out, int32_t count) {
  lbdd::g_err.clear();
  if (!ratio_out) return fail(LBDD_E_INVAL, "ratio_out is NULL");
  if (iters < 1) return fail(LBDD_E_INVAL, "iters < 1");
  if (count < 0 || (count > 0 && !ms_out)) return fail(LBDD_E_INVAL, "ms_out/count");
  static const int64_t CAND[] = {lbdd::SEARCH_RATIO_AUTO, 0, 64, lbdd::MAX_SEARCH_RATIO};
  constexpr int NC = sizeof(CAND) / sizeof(CAND[0]);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  Timer tm;
  if (hipError_t e = tm.init(); e != hipSuccess) return hip_err(e, "hipEventCreate");
  float times[NC] = {};
  int64_t obj0 = 0;
  for (int c = 0; c < NC; ++c) {
    lbdd_instance *h = nullptr;
    int rc = lbdd_create(k, n, cm, capacity, penalty, flags, hip_stream, &h);
    if (rc != LBDD_OK) return rc;
    rc = lbdd_set_option(h, LBDD_OPT_SEARCH_RATIO, CAND[c]);
    hipError_t e = hipSuccess;
    if (rc == LBDD_OK) e = hipEventRecord(tm.a, st);
    if (rc == LBDD_OK && e == hipSuccess) rc = lbdd_solve_iters(h, iters);
    if (rc == LBDD_OK && e == hipSuccess) e = hipEventRecord(tm.b, st);
    if (rc == LBDD_OK && e == hipSuccess) e = hipEventSynchronize(tm.b);
    float ms = 0.f;
    if (rc == LBDD_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, tm.a, tm.b);
    int64_t obj = 0;
    if (rc == LBDD_OK && e == hipSuccess) rc = lbdd_objective(h, &obj);
    lbdd_destroy(h);
    if (e != hipSuccess) return hip_err(e, "timing a candidate");
    if (rc != LBDD_OK) return rc;
    if (c == 0) obj0 = obj;
    else if (obj != obj0)   // every candidate computes the same allotment
      return fail(LBDD_E_INTERNAL, "search ratio %lld changed the objective", (long long)CAND[c]);
    if (c < count) ms_out[c] = ms;
    times[c] = ms;
  }
  // the default stays unless a candidate is faster by more than the noise
  int best = 0;
  while (CAND[best] != lbdd::DEFAULT_SEARCH_RATIO) ++best;
  const float base = times[best];
  for (int c = 0; c < NC; ++c)
    if (times[c] < NOISE * base && times[c] < times[best]) best = c;
  {
    std::lock_guard<std::mutex> g(lbdd::g_mu);
    lbdd::g_ratio[{lbdd::tune_bucket_k(k), lbdd::tune_bucket_n(n)}] = CAND[best];
  }
  *ratio_out = CAND[best];
  return NC;
}

int lbdd_tune_best_transfers(int32_t k, int64_t n, const int32_t *cm, const int32_t *assign,
                             const int32_t *rank, uint64_t *W, void *work, int32_t reps,
                             void *hip_stream, int32_t *config_out, float *ms_out) {
  lbdd::g_err.clear();
  if (k < 1 || k > LBDD_MAX_K) return fail(LBDD_E_INVAL, "k=%d outside [1, %d]", k, LBDD_MAX_K);
  if (n < 1 || n > LBDD_MAX_N) return fail(LBDD_E_INVAL, "n=%lld outside [1, 2^31-1]", (long long)n);
  if (!cm || !assign || !rank || !W || !work || !config_out || !ms_out)
    return fail(LBDD_E_INVAL, "NULL argument");
  if (reps < 1) return fail(LBDD_E_INVAL, "reps < 1");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const bool vec4 = lbdd::scan_vec4_ok(k, cm);
  lbdd::ScanCfg cand[64];
  const int nc = lbdd::scan_candidates(k, vec4, cand, 64);
  Timer tm;
  if (hipError_t e = tm.init(); e != hipSuccess) return hip_err(e, "hipEventCreate");
  // the default configuration's table, which every other one must reproduce
  uint64_t *ref = nullptr;
  int32_t *flag = nullptr;
  const int64_t kk = (int64_t)k * k;
  struct Free {
    hipStream_t st;
    void *p[2];
    ~Free() {
      for (void *q : p)
        if (q) (void)hipFreeAsync(q, st);
      (void)hipStreamSynchronize(st);
    }
  } guard{st, {nullptr, nullptr}};
  if (hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&ref), kk * 8, st); e != hipSuccess)
    return hip_err(e, "device allocation");
  guard.p[0] = ref;
  if (hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&flag), 4, st); e != hipSuccess)
    return hip_err(e, "device allocation");
  guard.p[1] = flag;
  const int32_t zero = 0;
  if (hipError_t e = hipMemcpyAsync(flag, &zero, 4, hipMemcpyHostToDevice, st); e != hipSuccess)
    return hip_err(e, "clear flag");
  int best = 0;
  float best_ms = 0.f, default_ms = 0.f;
  for (int c = 0; c < nc; ++c) {
    float total = 0.f;
    for (int r = 0; r <= reps; ++r) {   // the first run warms up
      // grouping once, W cleared before every timed pass
      hipError_t e = lbdd::launch_scan_group(k, n, assign, rank, W, work, c == 0 && r == 0, st);
      if (e == hipSuccess) e = hipEventRecord(tm.a, st);
      if (e == hipSuccess) e = lbdd::launch_scan_only(k, cm, work, cand[c], W, st);
      if (e == hipSuccess) e = hipEventRecord(tm.b, st);
      if (e == hipSuccess) e = hipEventSynchronize(tm.b);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, tm.a, tm.b);
      if (e != hipSuccess) return hip_err(e, "timing a scan configuration");
      if (r > 0) total += ms;
    }
    hipError_t e = c == 0 ? hipMemcpyAsync(ref, W, kk * 8, hipMemcpyDeviceToDevice, st)
                          : lbdd::launch_differ(ref, W, kk, flag, st);
    if (e != hipSuccess) return hip_err(e, "checking a scan configuration");
    const float ms = total / reps;
    if (c == 0) default_ms = best_ms = ms;   // candidate 0 is the default
    else if (ms < NOISE * default_ms && ms < best_ms) { best = c; best_ms = ms; }
  }
  int32_t differ = 0;
  hipError_t e0 = hipMemcpyAsync(&differ, flag, 4, hipMemcpyDeviceToHost, st);
  if (e0 == hipSuccess) e0 = hipStreamSynchronize(st);
  if (e0 != hipSuccess) return hip_err(e0, "checking the scan configurations");
  if (differ) return fail(LBDD_E_INTERNAL, "scan configurations disagree on the table");
  lbdd::scan_set_tuned(k, vec4, cand[best]);
  config_out[0] = cand[best].vec;
  config_out[1] = cand[best].lpr;
  config_out[2] = cand[best].np;
  config_out[3] = cand[best].mult;
  ms_out[0] = default_ms;
  ms_out[1] = best_ms;
  // leave W holding the table of the inputs, as lbdd_best_transfers would
  hipError_t e = lbdd::launch_scan_group(k, n, assign, rank, W, work, false, st);
  if (e == hipSuccess) e = lbdd::launch_scan_only(k, cm, work, cand[best], W, st);
  if (e != hipSuccess) return hip_err(e, "scan");
  return nc;
}


// ---- tuning cache ---------------------------------------------------------
// JSON: {"format": "lbdd-tune-1", "entries": [ {"arch": .., "kind": "search",
// "k_bucket": .., "n_bucket": .., "ratio": ..} | {"arch": .., "kind": "scan",
// "k": .., "vec4": 0|1, "config": [vec, lpr, np, mult]} ... ]}

}  // extern "C"

namespace {

// the part of the current device's architecture name before any feature
// suffix (gfx950:sramecc+:xnack- -> gfx950)
bool device_arch(std::string *out) {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return false;
  std::string a = p.gcnArchName;
  const size_t c = a.find(':');
  *out = c == std::string::npos ? a : a.substr(0, c);
  return !out->empty();
}

}  // namespace

extern "C" {

int lbdd_tune_save(const char *path, const char *arch) {
  lbdd::g_err.clear();
  if (!path) return fail(LBDD_E_INVAL, "path is NULL");
  std::string a;
  if (arch) a = arch;
  else if (!device_arch(&a)) return fail(LBDD_E_DEVICE, "cannot read the device architecture");
  if (a.empty() || a.find_first_of("\\\"") != std::string::npos) return fail(LBDD_E_INVAL, "bad arch name");
  std::vector<std::pair<std::pair<int, int>, int64_t>> search;
  {
    std::lock_guard<std::mutex> g(lbdd::g_mu);
    for (const auto &kv : lbdd::g_ratio) search.push_back(kv);
  }
  const std::vector<lbdd::ScanTuned> scan = lbdd::scan_tuned_list();
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = fopen(tmp.c_str(), "w");
  if (!f) return fail(LBDD_E_INVAL, "cannot write %s", tmp.c_str());
  fprintf(f, "{\"format\": \"lbdd-tune-1\", \"entries\": [");
  bool first = true;
  for (const auto &e : search) {
    fprintf(f, "%s\n  {\"arch\": \"%s\", \"kind\": \"search\", \"k_bucket\": %d, \"n_bucket\": %d, \"ratio\": %lld}",
            first ? "" : ",", a.c_str(), e.first.first, e.first.second, (long long)e.second);
    first = false;
  }
  for (const auto &e : scan) {
    fprintf(f, "%s\n  {\"arch\": \"%s\", \"kind\": \"scan\", \"k\": %d, \"vec4\": %d, \"config\": [%d, %d, %d, %d]}",
            first ? "" : ",", a.c_str(), e.k, e.vec4 ? 1 : 0, e.cfg.vec, e.cfg.lpr, e.cfg.np, e.cfg.mult);
    first = false;
  }
  fprintf(f, "\n]}\n");
  const bool ok = fflush(f) == 0 && !ferror(f);
  if (fclose(f) != 0 || !ok || rename(tmp.c_str(), path) != 0) {
    (void)remove(tmp.c_str());
    return fail(LBDD_E_INVAL, "cannot write %s", path);
  }
  return (int)(search.size() + scan.size());
}

int lbdd_tune_load(const char *path, const char *arch) {
  using lbdd::json::JParser;
  using lbdd::json::JVal;
  using lbdd::json::jint;
  lbdd::g_err.clear();
  if (!path) return fail(LBDD_E_INVAL, "path is NULL");
  std::string a;
  if (arch) a = arch;
  else if (!device_arch(&a)) return fail(LBDD_E_DEVICE, "cannot read the device architecture");
  FILE *f = fopen(path, "rb");
  if (!f) return fail(LBDD_E_INVAL, "cannot read %s", path);
  std::string text;
  char buf[4096];
  size_t m;
  while ((m = fread(buf, 1, sizeof buf, f)) > 0 && text.size() < (16u << 20)) text.append(buf, m);
  fclose(f);
  JVal root;
  JParser ps{text.data(), text.data() + text.size()};
  if (!ps.value(&root)) return fail(LBDD_E_INVAL, "%s is not JSON", path);
  ps.ws();
  if (ps.p != ps.end || root.kind != JVal::OBJ) return fail(LBDD_E_INVAL, "%s is not a tuning cache", path);
  const JVal *fmt = root.get("format"), *ents = root.get("entries");
  if (!fmt || fmt->kind != JVal::STR || fmt->str != "lbdd-tune-1" || !ents || ents->kind != JVal::ARR)
    return fail(LBDD_E_INVAL, "%s is not a tuning cache (format lbdd-tune-1)", path);
  // every entry is checked before any is applied
  std::vector<std::pair<std::pair<int, int>, int64_t>> search;
  std::vector<lbdd::ScanTuned> scan;
  for (size_t i = 0; i < ents->arr.size(); ++i) {
    const JVal &e = ents->arr[i];
    const JVal *ea = e.get("arch"), *kind = e.get("kind");
    if (e.kind != JVal::OBJ || !ea || ea->kind != JVal::STR || !kind || kind->kind != JVal::STR)
      return fail(LBDD_E_INVAL, "entry %zu: arch and kind needed", i);
    if (ea->str != a) continue;                  // tuned on another architecture
    if (kind->str == "search") {
      int64_t kb, nb, r;
      if (!jint(e.get("k_bucket"), 1, 12, &kb) || !jint(e.get("n_bucket"), 0, 10, &nb) ||
          !jint(e.get("ratio"), lbdd::SEARCH_RATIO_AUTO, lbdd::MAX_SEARCH_RATIO, &r))
        return fail(LBDD_E_INVAL, "entry %zu: bad search entry", i);
      search.push_back({{(int)kb, (int)nb}, r});
    } else if (kind->str == "scan") {
      int64_t k, v4, c[4];
      const JVal *cfg = e.get("config");
      bool ok = jint(e.get("k"), 1, LBDD_MAX_K, &k) && jint(e.get("vec4"), 0, 1, &v4) && cfg &&
                cfg->kind == JVal::ARR && cfg->arr.size() == 4;
      for (int j = 0; ok && j < 4; ++j) ok = jint(&cfg->arr[j], 1, 64, &c[j]);
      const lbdd::ScanCfg sc{(int32_t)c[0], (int32_t)c[1], (int32_t)c[2], (int32_t)c[3]};
      if (!ok || sc.vec != (v4 ? 4 : 1) || !lbdd::scan_cfg_valid((int32_t)k, sc))
        return fail(LBDD_E_INVAL, "entry %zu: bad scan entry", i);
      scan.push_back(lbdd::ScanTuned{(int32_t)k, v4 != 0, sc});
    } else {
      return fail(LBDD_E_INVAL, "entry %zu: unknown kind", i);
    }
  }
  {
    std::lock_guard<std::mutex> g(lbdd::g_mu);
    for (const auto &e : search) lbdd::g_ratio[e.first] = e.second;
  }
  for (const auto &e : scan) lbdd::scan_set_tuned(e.k, e.vec4, e.cfg);
  return (int)(search.size() + scan.size());
}

void lbdd_tune_clear(void) {
  {
    std::lock_guard<std::mutex> g(lbdd::g_mu);
    lbdd::g_ratio.clear();
  }
  lbdd::scan_clear_tuned();
}

}  // extern "C"
